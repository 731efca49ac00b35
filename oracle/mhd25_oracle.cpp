// mhd25_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, FP64 CPU reference ("oracle") for the Strang-split 2.5D ideal-MHD
// scheme of Fan & Fu, "Structure-preserving operator splitting for 2.5D ideal MHD
// with an entropy-stable DGSEM and exactly divergence-free compatible finite
// elements".  Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this library; the product path never does.  It shares no
// source, header or table generator with the HIP library.
//
// Every routine follows the paper's definitions in the paper's order, with
// deliberately literal loops (full double sums, explicit quadrature, normal
// equations solved by Gaussian elimination).  Readings of points the paper leaves
// open are marked "reading Rn" and are listed in the design notes.
//
// Layouts (identical to the C ABI so the same host arrays feed both sides):
//   U[5][K][p+1][p+1]    conservative (rho, m_x, m_y, m_z, E_mech) at GLL_p nodes,
//                        element e = ey*nx + ex, x index fastest;
//   rho, e: [K][p+1][p+1]; u: [3][K][p+1][p+1];
//   every magnetic array (B_x, B_y, B_z, E_*, J_*) is a periodic grid
//   [ny*(m+1)][nx*(m+1)] of physical nodal values (see node_* helpers below).
// Mirror walls (section "MHD rotor", reading R30): with bit 0 (bit 1) of walls set the mesh is the
// mirror-doubled image, in x (y), of the box formed by the first nx/2 (ny/2) elements of each row
// (column); every operator stays periodic on the doubled mesh and only the stabilisers' amplitudes
// (line_stats, B_global_amp) are taken over the box.
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cplx;

static inline double re(double x) { return x; }
static inline double re(const cplx& x) { return x.real(); }
// |x| and max() for the complex-step JVP take the branch of the real part.
static inline double absb(double x) { return std::fabs(x); }
static inline cplx absb(const cplx& x) { return x.real() < 0 ? -x : x; }
template <class T> static inline T maxb(const T& a, const T& b) { return re(a) >= re(b) ? a : b; }

// ---------------------------------------------------------------------------
// Section "Nodal bases, quadrature, and mass matrices": 1D rules and bases.
// ---------------------------------------------------------------------------

// Legendre polynomial P_n(x) and its first derivative by the three-term recurrence.
static void legendre(int n, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1; p1 = p2;
  }
  *P = p1;
  // derivative from the standard identity (x^2-1) P_n' = n (x P_n - P_{n-1})
  if (std::fabs(std::fabs(x) - 1.0) < 1e-300) {
    *dP = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
  } else {
    *dP = n * (x * p1 - p0) / (x * x - 1.0);
  }
}

// Gauss-Legendre rule with n points: nodes are the roots of P_n.
static void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0); w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double z = -std::cos(M_PI * (k + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP; legendre(n, z, &P, &dP);
      double dz = P / dP; z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double P, dP; legendre(n, z, &P, &dP);
    x[k] = z; w[k] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

// Gauss-Lobatto-Legendre rule of degree r (r+1 points): -1, 1 and the roots of
// P_r'; weights 2/(r(r+1)P_r(x)^2).  Degree 0 is the midpoint rule with weight 2.
static void gll_rule(int r, std::vector<double>& x, std::vector<double>& w) {
  x.assign(r + 1, 0.0); w.assign(r + 1, 0.0);
  if (r == 0) { x[0] = 0.0; w[0] = 2.0; return; }
  x[0] = -1.0; x[r] = 1.0;
  for (int k = 1; k < r; ++k) {
    double z = -std::cos(M_PI * k / r);
    for (int it = 0; it < 100; ++it) {
      double P, dP; legendre(r, z, &P, &dP);
      // (1-z^2) P'' = 2 z P' - r(r+1) P
      double d2P = (2.0 * z * dP - r * (r + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P; z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[k] = z;
  }
  for (int k = 0; k <= r; ++k) {
    double P, dP; legendre(r, x[k], &P, &dP);
    w[k] = 2.0 / (r * (r + 1.0) * P * P);
  }
}

// Lagrange basis function j of the node set xs, and its derivative, at x.
static double lag(const std::vector<double>& xs, int j, double x) {
  double v = 1.0;
  for (size_t k = 0; k < xs.size(); ++k)
    if ((int)k != j) v *= (x - xs[k]) / (xs[j] - xs[k]);
  return v;
}
static double dlag(const std::vector<double>& xs, int j, double x) {
  double s = 0.0;
  for (size_t l = 0; l < xs.size(); ++l) {
    if ((int)l == j) continue;
    double t = 1.0 / (xs[j] - xs[l]);
    for (size_t k = 0; k < xs.size(); ++k)
      if ((int)k != j && k != l) t *= (x - xs[k]) / (xs[j] - xs[k]);
    s += t;
  }
  return s;
}

// Dense solve A x = b (n x n, row major) by Gaussian elimination with partial pivoting.
static void gsolve(int n, std::vector<double> A, std::vector<double>& b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = b[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
    b[c] = s / A[c * n + c];
  }
}

// r-th derivative of P_a at x = +1 and x = -1 (closed form (a+r)!/(2^r r!(a-r)!)).
static double dleg_end(int a, int r, int side /*+1 or -1*/) {
  if (r > a) return 0.0;
  double v = 1.0;
  for (int k = a - r + 1; k <= a + r; ++k) v *= k;
  for (int k = 1; k <= r; ++k) v /= 2.0 * k;
  if (side < 0 && ((a + r) % 2)) v = -v;
  return v;
}

// ---------------------------------------------------------------------------
// Mesh, tables and node maps.
// ---------------------------------------------------------------------------
struct Mesh {
  int nx, ny, p, m;
  int walls;   // bit 0 / bit 1: mirror-doubled in x / y (statistics over the box)
  int bx, by;  // elements per row / column of the box the statistics cover
  double x0, x1, y0, y1, gamma, hx, hy, J;  // J = |J_K| = hx*hy/4
  int np;      // (p+1)
  int nn;      // (p+1)^2 nodes per element
  int M1;      // m+1
  long K;
  std::vector<double> xi, om;     // GLL_p
  std::vector<double> xw, ow;     // GLL_{m+1}  (m+2 points)
  std::vector<double> zg, og;     // Gauss_m    (m+1 points)
  std::vector<double> xv, ov;     // GLL_m      (m+1 points; midpoint for m=0)
  std::vector<double> zq, oq;     // Gauss_{m+1}(m+2 points), exact rule for the RT block
  std::vector<double> Dm;         // D_ij = l_j'(xi_i) on GLL_p
};
struct Opts {
  int oe_hydro, oe_mag, pp, ar, iface_flux, max_halvings;
  int strang_order;  // 0: H(dt/2) M(dt) H(dt/2), 1: M(dt/2) H(dt) M(dt/2)
  double sH, sM, Cs, Ceta;
};

static Mesh make_mesh(const int* im, const double* dm) {
  Mesh M;
  M.nx = im[0]; M.ny = im[1]; M.p = im[2]; M.m = im[3]; M.walls = im[4];
  M.bx = (M.walls & 1) ? M.nx / 2 : M.nx; M.by = (M.walls & 2) ? M.ny / 2 : M.ny;
  M.x0 = dm[0]; M.x1 = dm[1]; M.y0 = dm[2]; M.y1 = dm[3]; M.gamma = dm[4];
  M.hx = (M.x1 - M.x0) / M.nx; M.hy = (M.y1 - M.y0) / M.ny; M.J = M.hx * M.hy / 4.0;
  M.np = M.p + 1; M.nn = M.np * M.np; M.M1 = M.m + 1; M.K = (long)M.nx * M.ny;
  gll_rule(M.p, M.xi, M.om);
  gll_rule(M.m + 1, M.xw, M.ow);
  gauss_rule(M.m + 1, M.zg, M.og);
  gll_rule(M.m, M.xv, M.ov);
  gauss_rule(M.m + 2, M.zq, M.oq);
  M.Dm.assign(M.nn, 0.0);
  for (int i = 0; i < M.np; ++i)
    for (int j = 0; j < M.np; ++j) M.Dm[i * M.np + j] = dlag(M.xi, j, M.xi[i]);
  return M;
}
static Opts make_opts(const int* io, const double* dop) {
  Opts o;
  o.oe_hydro = io[0]; o.oe_mag = io[1]; o.pp = io[2]; o.ar = io[3];
  o.iface_flux = io[4]; o.max_halvings = io[5]; o.strang_order = io[6];
  o.sH = dop[0]; o.sM = dop[1]; o.Cs = dop[2]; o.Ceta = dop[3];
  return o;
}

static inline long emod(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }
static inline long elem(const Mesh& M, long ex, long ey) { return emod(ey, M.ny) * M.nx + emod(ex, M.nx); }
// node (i,j) of element e in a [.][K][p+1][p+1] array of component c
static inline long nid(const Mesh& M, int c, long e, int i, int j) {
  return ((long)c * M.K + e) * M.nn + (long)j * M.np + i;
}
// global index of a magnetic grid node: element (ex,ey), local (i,j), with the
// last GLL_{m+1} node (local index m+1) wrapping onto the next element's node 0.
static inline long gid(const Mesh& M, long ex, long ey, int i, int j) {
  long gx = emod(ex * M.M1 + i, (long)M.nx * M.M1);
  long gy = emod(ey * M.M1 + j, (long)M.ny * M.M1);
  return gy * (long)M.nx * M.M1 + gx;
}

// ---------------------------------------------------------------------------
// Section "Hydrodynamic subflow": Euler state, physical fluxes, EC and LLF fluxes.
// ---------------------------------------------------------------------------
template <class T> struct St { T r, mx, my, mz, E; };

template <class T> static inline T pressure(const St<T>& s, double g) {
  return (g - 1.0) * (s.E - (s.mx * s.mx + s.my * s.my + s.mz * s.mz) / (2.0 * s.r));
}

// physical Euler flux F_d(U), d = 0 (x) or 1 (y)
template <class T> static void phys_flux(const St<T>& s, int d, double g, T* F) {
  T ux = s.mx / s.r, uy = s.my / s.r;
  T p = pressure(s, g);
  T ud = d == 0 ? ux : uy;
  F[0] = d == 0 ? s.mx : s.my;
  F[1] = s.mx * ud + (d == 0 ? p : T(0.0));
  F[2] = s.my * ud + (d == 1 ? p : T(0.0));
  F[3] = s.mz * ud;
  F[4] = (s.E + p) * ud;
}

// logarithmic mean a^log = (aR-aL)/(log aR - log aL), continuous extension aL.
// Written through f = (aR-aL)/(aR+aL): a^log = {{a}} * f / atanh(f); for small f
// the textbook series f/atanh f = 1/(1 + f^2/3 + f^4/5 + ...) is summed far past
// double precision, otherwise the quotient is taken with log(aR/aL).
template <class T> static T logmean(const T& aL, const T& aR) {
  T f = (aR - aL) / (aR + aL);
  if (std::fabs(re(f)) < 0.05) {
    T u = f * f, s = T(0.0);
    for (int k = 10; k >= 1; --k) s = s * u + T(1.0 / (2.0 * k + 1.0));
    s = s * u + T(1.0);
    return 0.5 * (aL + aR) / s;
  }
  return (aR - aL) / std::log(aR / aL);
}

// Chandrashekar entropy-conservative flux, 2.5D form (eq. euler-chandrashekar-flux).
template <class T> static void ec_flux(const St<T>& L, const St<T>& R, int d, double g, T* F) {
  T uxL = L.mx / L.r, uyL = L.my / L.r, uzL = L.mz / L.r;
  T uxR = R.mx / R.r, uyR = R.my / R.r, uzR = R.mz / R.r;
  T pL = pressure(L, g), pR = pressure(R, g);
  T bL = L.r / (2.0 * pL), bR = R.r / (2.0 * pR);
  T rlog = logmean(L.r, R.r), blog = logmean(bL, bR);
  T ra = 0.5 * (L.r + R.r), ba = 0.5 * (bL + bR);
  T uxa = 0.5 * (uxL + uxR), uya = 0.5 * (uyL + uyR), uza = 0.5 * (uzL + uzR);
  T u2a = 0.5 * ((uxL * uxL + uyL * uyL + uzL * uzL) + (uxR * uxR + uyR * uyR + uzR * uzR));
  T phat = ra / (2.0 * ba);
  T hhat = 1.0 / (2.0 * (g - 1.0) * blog) - 0.5 * u2a + (uxa * uxa + uya * uya + uza * uza) + phat / rlog;
  T ud = d == 0 ? uxa : uya;
  F[0] = rlog * ud;
  F[1] = rlog * uxa * ud + (d == 0 ? phat : T(0.0));
  F[2] = rlog * uya * ud + (d == 1 ? phat : T(0.0));
  F[3] = rlog * uza * ud;
  F[4] = rlog * ud * hhat;
}

// local Lax-Friedrichs interface flux (eq. euler-lf-flux)
template <class T> static void llf_flux(const St<T>& Lm, const St<T>& Rp, int d, double g, T* F) {
  T FL[5], FR[5];
  phys_flux(Lm, d, g, FL); phys_flux(Rp, d, g, FR);
  T udL = (d == 0 ? Lm.mx : Lm.my) / Lm.r, udR = (d == 0 ? Rp.mx : Rp.my) / Rp.r;
  T cL = std::sqrt(g * pressure(Lm, g) / Lm.r), cR = std::sqrt(g * pressure(Rp, g) / Rp.r);
  T lam = maxb(absb(udL) + cL, absb(udR) + cR);
  T dU[5] = {Rp.r - Lm.r, Rp.mx - Lm.mx, Rp.my - Lm.my, Rp.mz - Lm.mz, Rp.E - Lm.E};
  for (int c = 0; c < 5; ++c) F[c] = 0.5 * (FL[c] + FR[c]) - 0.5 * lam * dU[c];
}

template <class T> static inline St<T> load_state(const Mesh& M, const T* U, long e, int i, int j) {
  St<T> s;
  s.r = U[nid(M, 0, e, i, j)]; s.mx = U[nid(M, 1, e, i, j)]; s.my = U[nid(M, 2, e, i, j)];
  s.mz = U[nid(M, 3, e, i, j)]; s.E = U[nid(M, 4, e, i, j)];
  return s;
}

// L_E: mass-inverted DGSEM operator, eq. euler-nodal-index evaluated literally
// (full double sum of eq. euler-volume-residual, boundary corrections at i,j in {0,p}).
template <class T> static void rhs_hydro_t(const Mesh& M, int iface_flux, const T* U, T* dU) {
  const int p = M.p, np = M.np;
  const double g = M.gamma;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    long eL = elem(M, ex - 1, ey), eR = elem(M, ex + 1, ey);
    long eB = elem(M, ex, ey - 1), eT = elem(M, ex, ey + 1);
    for (int j = 0; j < np; ++j)
      for (int i = 0; i < np; ++i) {
        St<T> Ui = load_state(M, U, e, i, j);
        T R[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)}, F[5];
        for (int r = 0; r < np; ++r) {  // x-direction volume term
          ec_flux(Ui, load_state(M, U, e, r, j), 0, g, F);
          double Q = M.om[i] * M.Dm[i * np + r];
          for (int c = 0; c < 5; ++c) R[c] += 2.0 * Q * M.om[j] * (M.hy / 2.0) * F[c];
        }
        for (int s = 0; s < np; ++s) {  // y-direction volume term
          ec_flux(Ui, load_state(M, U, e, i, s), 1, g, F);
          double Q = M.om[j] * M.Dm[j * np + s];
          for (int c = 0; c < 5; ++c) R[c] += 2.0 * M.om[i] * Q * (M.hx / 2.0) * F[c];
        }
        T Fp[5], Fs[5];
        auto num = [&](const St<T>& a, const St<T>& b, int d, T* out) {
          if (iface_flux == 1) ec_flux(a, b, d, g, out); else llf_flux(a, b, d, g, out);
        };
        if (i == 0) {  // left face: U^- from the left neighbour, U^+ = own trace
          phys_flux(Ui, 0, g, Fp); num(load_state(M, U, eL, p, j), Ui, 0, Fs);
          for (int c = 0; c < 5; ++c) R[c] += M.om[j] * (M.hy / 2.0) * (Fp[c] - Fs[c]);
        }
        if (i == p) {
          phys_flux(Ui, 0, g, Fp); num(Ui, load_state(M, U, eR, 0, j), 0, Fs);
          for (int c = 0; c < 5; ++c) R[c] -= M.om[j] * (M.hy / 2.0) * (Fp[c] - Fs[c]);
        }
        if (j == 0) {
          phys_flux(Ui, 1, g, Fp); num(load_state(M, U, eB, i, p), Ui, 1, Fs);
          for (int c = 0; c < 5; ++c) R[c] += M.om[i] * (M.hx / 2.0) * (Fp[c] - Fs[c]);
        }
        if (j == p) {
          phys_flux(Ui, 1, g, Fp); num(Ui, load_state(M, U, eT, i, 0), 1, Fs);
          for (int c = 0; c < 5; ++c) R[c] -= M.om[i] * (M.hx / 2.0) * (Fp[c] - Fs[c]);
        }
        double Mij = M.J * M.om[i] * M.om[j];
        for (int c = 0; c < 5; ++c) dU[nid(M, c, e, i, j)] = -R[c] / Mij;
      }
  }
}

// ---------------------------------------------------------------------------
// Oscillation elimination (section "Oscillation-eliminating procedure").
// ---------------------------------------------------------------------------

// Projections Pi^l (l = 0..p) of one element's nodal field w under a weighted
// GLL product sum_q W_q v_q z_q onto Q^l, each solved from its own normal
// equations in the tensor Legendre basis.  out[l][q] = (Pi^l w)(x_q).
static void projections(const Mesh& M, const double* w, const double* W, std::vector<double>& out) {
  const int np = M.np, nn = M.nn;
  std::vector<double> Lv(np * np);  // Lv[a*np+i] = P_a(xi_i)
  for (int a = 0; a < np; ++a)
    for (int i = 0; i < np; ++i) { double P, dP; legendre(a, M.xi[i], &P, &dP); Lv[a * np + i] = P; }
  out.assign((size_t)np * nn, 0.0);
  for (int l = 0; l < np; ++l) {
    int nb = (l + 1) * (l + 1);
    std::vector<double> G(nb * nb, 0.0), b(nb, 0.0), phi((size_t)nb * nn);
    for (int a = 0, k = 0; a <= l; ++a)
      for (int bb = 0; bb <= l; ++bb, ++k)
        for (int j = 0; j < np; ++j)
          for (int i = 0; i < np; ++i) phi[(size_t)k * nn + j * np + i] = Lv[a * np + i] * Lv[bb * np + j];
    for (int k = 0; k < nb; ++k) {
      for (int k2 = 0; k2 < nb; ++k2) {
        double s = 0.0;
        for (int q = 0; q < nn; ++q) s += W[q] * phi[(size_t)k * nn + q] * phi[(size_t)k2 * nn + q];
        G[k * nb + k2] = s;
      }
      double s = 0.0;
      for (int q = 0; q < nn; ++q) s += W[q] * phi[(size_t)k * nn + q] * w[q];
      b[k] = s;
    }
    gsolve(nb, G, b);
    for (int q = 0; q < nn; ++q) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += b[k] * phi[(size_t)k * nn + q];
      out[(size_t)l * nn + q] = s;
    }
  }
}

// Physical derivatives of orders r = 0..p of the element polynomial of w along the
// nodal line `line` (dir 0: x-line at fixed y-node, dir 1: y-line at fixed x-node),
// evaluated at the end side (-1 or +1).  The 1D interpolant is expanded in
// Legendre polynomials (Vandermonde solve) and differentiated in closed form.
static void line_end_derivs(const Mesh& M, const double* w_elem, int dir, int line, int side, double* out) {
  const int np = M.np;
  std::vector<double> V(np * np), c(np);
  for (int i = 0; i < np; ++i) {
    for (int a = 0; a < np; ++a) { double P, dP; legendre(a, M.xi[i], &P, &dP); V[i * np + a] = P; }
    c[i] = dir == 0 ? w_elem[line * np + i] : w_elem[i * np + line];
  }
  gsolve(np, V, c);
  double h = dir == 0 ? M.hx : M.hy;
  for (int r = 0; r < np; ++r) {
    double s = 0.0;
    for (int a = 0; a < np; ++a) s += c[a] * dleg_end(a, r, side);
    out[r] = s * std::pow(2.0 / h, r);
  }
}

// Normal-jump measure J_{r,I,K}(w) (eq. euler-oe-jump) for all r = 0..p.
// Face integrals use the element's GLL_p face nodes: (1/|F|) int_F f = 1/2 sum_k om_k f_k
// (reading R10).  `field(e)` returns element e's nodal values.
template <class FieldFn>
static void jump_measure(const Mesh& M, long e, int dir, FieldFn field, double* Jr) {
  long ex = e % M.nx, ey = e / M.nx;
  long em = dir == 0 ? elem(M, ex - 1, ey) : elem(M, ex, ey - 1);
  long ep = dir == 0 ? elem(M, ex + 1, ey) : elem(M, ex, ey + 1);
  const double* w = field(e);
  const double* wm = field(em);
  const double* wp = field(ep);
  std::vector<double> sm(M.np, 0.0), sp(M.np, 0.0), a(M.np), b(M.np), c(M.np), d(M.np);
  for (int k = 0; k < M.np; ++k) {
    line_end_derivs(M, w, dir, k, -1, a.data());
    line_end_derivs(M, wm, dir, k, +1, b.data());
    line_end_derivs(M, wp, dir, k, -1, c.data());
    line_end_derivs(M, w, dir, k, +1, d.data());
    for (int r = 0; r <= M.p; ++r) {
      double jm = a[r] - b[r], jp = c[r] - d[r];
      sm[r] += 0.5 * M.om[k] * jm * jm;
      sp[r] += 0.5 * M.om[k] * jp * jp;
    }
  }
  for (int r = 0; r <= M.p; ++r) Jr[r] = std::sqrt(sm[r]) + std::sqrt(sp[r]);
}

// Global and cross-line statistics of a nodal scalar field (eq. euler-oe-amplitude).
// Means use the GLL quadrature (reading R9).  Outputs per field:
//   dOm = Delta_Omega(w); rowD[ey] = Delta_{x,K} for elements of row ey; colD[ex] = Delta_{y,K};
//   const_flag = 1 if the field is constant to roundoff (reading R11).
struct LineStats { double dOm; std::vector<double> rowD, colD; int const_flag; };

// With mirror walls every sum, mean and extremum runs over the box: its elements, and for a row
// (column) the row's (column's) first bx (by) elements.
static bool in_box(const Mesh& M, long e) { return e % M.nx < M.bx && e / M.nx < M.by; }

static LineStats line_stats(const Mesh& M, const double* w /*[K][nn]*/) {
  LineStats S;
  double sum = 0.0, area = 0.0, amax = 0.0;
  for (long e = 0; e < M.K; ++e) {
    if (!in_box(M, e)) continue;
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) {
        double v = w[e * M.nn + j * M.np + i];
        sum += M.J * M.om[i] * M.om[j] * v;
        amax = std::max(amax, std::fabs(v));
      }
  }
  area = (double)M.bx * M.by * M.hx * M.hy;
  double mean = sum / area;
  double d = 0.0, vmin = w[0], vmax = w[0];
  for (long q = 0; q < M.K * M.nn; ++q) {
    if (!in_box(M, q / M.nn)) continue;
    d = std::max(d, std::fabs(w[q] - mean));
    vmin = std::min(vmin, w[q]); vmax = std::max(vmax, w[q]);
  }
  S.dOm = d;
  // constant to roundoff: the nodal values agree to 2^10 ulps of the field's size (an exact test,
  // independent of how the mean was summed)
  S.const_flag = vmax - vmin <= 1024.0 * 2.220446049250313e-16 * amax ? 1 : 0;
  S.rowD.assign(M.ny, 0.0); S.colD.assign(M.nx, 0.0);
  for (int pass = 0; pass < 2; ++pass) {
    int nl = pass == 0 ? M.ny : M.nx, len = pass == 0 ? M.bx : M.by;
    for (int l = 0; l < nl; ++l) {
      double s = 0.0, a = 0.0;
      for (int t = 0; t < len; ++t) {
        long e = pass == 0 ? (long)l * M.nx + t : (long)t * M.nx + l;
        for (int j = 0; j < M.np; ++j)
          for (int i = 0; i < M.np; ++i) s += M.J * M.om[i] * M.om[j] * w[e * M.nn + j * M.np + i];
        a += M.hx * M.hy;
      }
      double lm = s / a, dl = 0.0;
      for (int t = 0; t < len; ++t) {
        long e = pass == 0 ? (long)l * M.nx + t : (long)t * M.nx + l;
        for (int q = 0; q < M.nn; ++q) dl = std::max(dl, std::fabs(w[e * M.nn + q] - lm));
      }
      dl = std::max(dl, 1e-6 * d);
      (pass == 0 ? S.rowD : S.colD)[l] = dl;
    }
  }
  return S;
}

static double factorial(int r) { double f = 1.0; for (int k = 2; k <= r; ++k) f *= k; return f; }

// Shared-amplitude sensor sigma_{r,I,K} of a set of nq scalar fields
// (eq. euler-oe-sigma, eq. magnetic-oe-sensor).  sig[dir][r].
static void oe_sensor(const Mesh& M, long e, int nq, const double* const* fields,
                      const std::vector<LineStats>& S, std::vector<double>& sig) {
  long ex = e % M.nx, ey = e / M.nx;
  sig.assign(2 * M.np, 0.0);
  for (int dir = 0; dir < 2; ++dir) {
    double Dsh = 0.0;  // shared amplitude: max over components
    for (int q = 0; q < nq; ++q) Dsh = std::max(Dsh, dir == 0 ? S[q].rowD[ey] : S[q].colD[ex]);
    if (!(Dsh > 0.0)) continue;
    double h = dir == 0 ? M.hx : M.hy;
    for (int q = 0; q < nq; ++q) {
      if (S[q].const_flag) continue;
      std::vector<double> Jr(M.np);
      const double* f = fields[q];
      jump_measure(M, e, dir, [&](long ee) { return f + ee * M.nn; }, Jr.data());
      for (int r = 0; r <= M.p; ++r) {
        double v = (2.0 * r + 1.0) * std::pow(h, r) / (2.0 * factorial(r)) * Jr[r] / Dsh;
        sig[dir * M.np + r] = std::max(sig[dir * M.np + r], v);
      }
    }
  }
}

// P_OE for the Euler state (eq. euler-oe-map); tau is the substep (reading R7).
static void hydro_oe(const Mesh& M, const Opts& o, double tau, const double* Uin, double* Uout, double* Dout) {
  const int nn = M.nn;
  std::vector<LineStats> S(5);
  for (int c = 0; c < 5; ++c) S[c] = line_stats(M, Uin + (long)c * M.K * nn);
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    const double* fields[5];
    for (int c = 0; c < 5; ++c) fields[c] = Uin + (long)c * M.K * nn;
    std::vector<double> sig;
    oe_sensor(M, e, 5, fields, S, sig);
    // cell average and direction-matched rate (eq. euler-oe-rate, reading R12)
    double avg[5];
    for (int c = 0; c < 5; ++c) {
      double s = 0.0;
      for (int j = 0; j < M.np; ++j)
        for (int i = 0; i < M.np; ++i) s += M.J * M.om[i] * M.om[j] * Uin[nid(M, c, e, i, j)];
      avg[c] = s / (M.hx * M.hy);
    }
    St<double> a{avg[0], avg[1], avg[2], avg[3], avg[4]};
    double cK = std::sqrt(M.gamma * pressure(a, M.gamma) / a.r);
    double lam[2] = {(2.0 * M.p + 1.0) * (std::fabs(a.mx / a.r) + cK) / M.hx,
                     (2.0 * M.p + 1.0) * (std::fabs(a.my / a.r) + cK) / M.hy};
    std::vector<double> D(M.np, 1.0);
    for (int l = 1; l <= M.p; ++l) {
      double Th = 0.0;
      for (int dir = 0; dir < 2; ++dir) {
        double s = 0.0;
        for (int r = 0; r <= l; ++r) s += sig[dir * M.np + r];
        Th += lam[dir] * s;
      }
      D[l] = std::exp(-o.sH * tau * Th);
    }
    if (Dout) for (int l = 0; l <= M.p; ++l) Dout[e * M.np + l] = D[l];
    std::vector<double> Wq(nn);
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) Wq[j * M.np + i] = M.J * M.om[i] * M.om[j];
    for (int c = 0; c < 5; ++c) {
      std::vector<double> Pi;
      projections(M, Uin + ((long)c * M.K + e) * nn, Wq.data(), Pi);
      for (int q = 0; q < nn; ++q) {
        double v = Pi[q];
        for (int l = 1; l <= M.p; ++l) v += D[l] * (Pi[(size_t)l * nn + q] - Pi[(size_t)(l - 1) * nn + q]);
        Uout[((long)c * M.K + e) * nn + q] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Positivity-preserving scaling (eq. euler-pp-floors .. euler-pp-pressure, reading R14).
// flags bit0: density limited, bit1: pressure limited, bit2: collapsed.
// ---------------------------------------------------------------------------
static const double EPS = 2.220446049250313e-16;  // 2^-52 (reading R1)

static void element_average(const Mesh& M, const double* U, long e, double* avg) {
  for (int c = 0; c < 5; ++c) {
    double s = 0.0;
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) s += M.J * M.om[i] * M.om[j] * U[nid(M, c, e, i, j)];
    avg[c] = s / (M.hx * M.hy);
  }
}

static uint8_t pp_element(const Mesh& M, double* U, long e) {
  const double g = M.gamma;
  const double eps_r = 64.0 * EPS;
  double avg[5];
  element_average(M, U, e, avg);
  St<double> a{avg[0], avg[1], avg[2], avg[3], avg[4]};
  double pbar = pressure(a, g);
  auto Sp = [&](const St<double>& s) {
    return std::fabs(s.E) + (s.mx * s.mx + s.my * s.my + s.mz * s.mz) / (2.0 * std::max(s.r, eps_r));
  };
  auto collapse = [&]() {
    for (int c = 0; c < 5; ++c)
      for (int q = 0; q < M.nn; ++q) U[((long)c * M.K + e) * M.nn + q] = avg[c];
    return (uint8_t)4;
  };
  if (a.r <= eps_r) return collapse();
  uint8_t flags = 0;
  double rmin = U[nid(M, 0, e, 0, 0)];
  for (int q = 0; q < M.nn; ++q) rmin = std::min(rmin, U[(long)e * M.nn + q]);
  if (rmin < eps_r) {
    double th = (a.r - eps_r) / (a.r - rmin);
    th = std::min(1.0, std::max(0.0, th));
    for (int q = 0; q < M.nn; ++q) {
      double& r = U[(long)e * M.nn + q];
      r = a.r + th * (r - a.r);
    }
    flags |= 1;
  }
  double S = Sp(a);
  for (int j = 0; j < M.np; ++j)
    for (int i = 0; i < M.np; ++i) S = std::max(S, Sp(load_state(M, U, e, i, j)));
  double eps_p = std::max(64.0 * EPS, 8192.0 * EPS * S);
  if (pbar <= eps_p) return (uint8_t)(flags | collapse());
  double pmin = pressure(load_state(M, U, e, 0, 0), g);
  for (int j = 0; j < M.np; ++j)
    for (int i = 0; i < M.np; ++i) pmin = std::min(pmin, pressure(load_state(M, U, e, i, j), g));
  if (pmin < eps_p) {
    double th = (pbar - eps_p) / (pbar - pmin);
    th = std::min(1.0, std::max(0.0, th));
    for (int c = 0; c < 5; ++c)
      for (int q = 0; q < M.nn; ++q) {
        double& v = U[((long)c * M.K + e) * M.nn + q];
        v = avg[c] + th * (v - avg[c]);
      }
    flags |= 2;
  }
  return flags;
}

// raw-average admissibility (section "SSP-RK(3,3) update"; NaN-safe, reading R14)
static bool averages_admissible(const Mesh& M, const double* U) {
  bool ok = true;
  for (long e = 0; e < M.K; ++e) {
    double avg[5];
    element_average(M, U, e, avg);
    St<double> a{avg[0], avg[1], avg[2], avg[3], avg[4]};
    if (!(a.r > 0.0) || !(pressure(a, M.gamma) > 0.0)) ok = false;
  }
  return ok;
}

// Stage map P = P_PP o P_OE (eq. euler-stage-map) applied to a raw candidate.
static void hydro_stage_map(const Mesh& M, const Opts& o, double tau, double* U, uint8_t* flags,
                            int64_t* counts, double* Dout) {
  const long n = 5 * M.K * M.nn;
  if (o.oe_hydro) {
    std::vector<double> tmp(n);
    hydro_oe(M, o, tau, U, tmp.data(), Dout);
    std::memcpy(U, tmp.data(), n * sizeof(double));
  }
  for (long e = 0; e < M.K; ++e) {
    uint8_t f = o.pp ? pp_element(M, U, e) : 0;
    if (flags) flags[e] = f;
    if (counts) { counts[0] += (f & 1) != 0; counts[1] += (f & 2) != 0; counts[2] += (f & 4) != 0; }
  }
}

// ---------------------------------------------------------------------------
// Admissibility of an input state: the admissible set of section "Conservative ideal MHD"
// (positive density and pressure) at every node, with every value finite.  An input outside
// it is refused with status 2 before anything is modified.
// ---------------------------------------------------------------------------
static bool all_finite(const double* a, long n) {
  for (long k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

static bool state_admissible(const Mesh& M, const double* U) {
  for (long e = 0; e < M.K; ++e)
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) {
        St<double> s = load_state(M, U, e, i, j);
        const double v[5] = {s.r, s.mx, s.my, s.mz, s.E};
        if (!all_finite(v, 5)) return false;
        if (!(s.r > 0.0) || !(pressure(s, M.gamma) > 0.0)) return false;
      }
  return true;
}

// the magnetic substep's state: rho > 0 and e > 0 (so p = (gamma - 1) rho e > 0), all finite
static bool primitive_admissible(const Mesh& M, const double* rho, const double* en, const double* u) {
  const long n = M.K * M.nn;
  if (!all_finite(u, 3 * n)) return false;
  for (long q = 0; q < n; ++q)
    if (!std::isfinite(rho[q]) || !std::isfinite(en[q]) || !(rho[q] > 0.0) || !(en[q] > 0.0)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Hydrodynamic substep (Algorithm "Hydrodynamic Euler substep", eq. euler-ssprk33)
// with reject-and-halve (reading R15: a rejected attempt is replaced by two
// attempts of half the step, recursively).
// ---------------------------------------------------------------------------
struct Report {
  int32_t attempted, accepted, max_depth, status;
  int64_t n_rho, n_p, n_col;
  double eta_max, dt;
};

static bool hydro_attempt(const Mesh& M, const Opts& o, double* U, double tau, uint8_t* flags, int64_t* counts) {
  const long n = 5 * M.K * M.nn;
  std::vector<double> Un(U, U + n), L(n), S1(n), S2(n), Y(n);
  int64_t c[3] = {0, 0, 0};
  rhs_hydro_t<double>(M, o.iface_flux, Un.data(), L.data());
  for (long q = 0; q < n; ++q) Y[q] = Un[q] + tau * L[q];
  if (!averages_admissible(M, Y.data())) return false;
  hydro_stage_map(M, o, tau, Y.data(), flags, c, nullptr);
  S1 = Y;
  rhs_hydro_t<double>(M, o.iface_flux, S1.data(), L.data());
  for (long q = 0; q < n; ++q) Y[q] = 0.75 * Un[q] + 0.25 * (S1[q] + tau * L[q]);
  if (!averages_admissible(M, Y.data())) return false;
  hydro_stage_map(M, o, tau, Y.data(), flags, c, nullptr);
  S2 = Y;
  rhs_hydro_t<double>(M, o.iface_flux, S2.data(), L.data());
  for (long q = 0; q < n; ++q) Y[q] = (1.0 / 3.0) * Un[q] + (2.0 / 3.0) * (S2[q] + tau * L[q]);
  if (!averages_admissible(M, Y.data())) return false;
  hydro_stage_map(M, o, tau, Y.data(), flags, c, nullptr);
  std::memcpy(U, Y.data(), n * sizeof(double));
  counts[0] += c[0]; counts[1] += c[1]; counts[2] += c[2];
  return true;
}

static int hydro_substep_rec(const Mesh& M, const Opts& o, double* U, double tau, int depth, Report* rep,
                             uint8_t* flags, int32_t* log, int log_cap) {
  rep->attempted++;
  rep->max_depth = std::max(rep->max_depth, depth);
  int64_t cnt[3] = {0, 0, 0};
  bool ok = hydro_attempt(M, o, U, tau, flags, cnt);
  if (log && rep->attempted <= log_cap) log[rep->attempted - 1] = depth * 2 + (ok ? 1 : 0);
  if (ok) {
    rep->accepted++;
    rep->n_rho += cnt[0]; rep->n_p += cnt[1]; rep->n_col += cnt[2];
    return 0;
  }
  if (depth + 1 > o.max_halvings) return 1;
  int s = hydro_substep_rec(M, o, U, 0.5 * tau, depth + 1, rep, flags, log, log_cap);
  if (s) return s;
  return hydro_substep_rec(M, o, U, 0.5 * tau, depth + 1, rep, flags, log, log_cap);
}

// ---------------------------------------------------------------------------
// Magnetic-velocity subflow (section "Magnetic--velocity subflow").
// Local node sets of element K (m = magnetic degree, M1 = m+1):
//   B_x, E_y, J_y : GLL_{m+1} (i = 0..m+1) in x  x  Gauss_m (j = 0..m) in y
//   B_y, E_x, J_x : Gauss_m (i = 0..m) in x       x  GLL_{m+1} (j = 0..m+1) in y
//   B_z           : GLL_m x GLL_m (i, j = 0..m), element-local
//   E_z, J_z      : GLL_{m+1} x GLL_{m+1} (i, j = 0..m+1)
// ---------------------------------------------------------------------------

// evaluate a tensor-product nodal field at reference point (X, Y)
template <class T>
static T eval_tensor(const std::vector<double>& nx_, const std::vector<double>& ny_, const T* vals /*[j][i]*/,
                     double X, double Y, int dx, int dy) {
  T s = T(0.0);
  for (size_t j = 0; j < ny_.size(); ++j) {
    double ly = dy ? dlag(ny_, (int)j, Y) : lag(ny_, (int)j, Y);
    for (size_t i = 0; i < nx_.size(); ++i) {
      double lx = dx ? dlag(nx_, (int)i, X) : lag(nx_, (int)i, X);
      s += vals[j * nx_.size() + i] * (lx * ly);
    }
  }
  return s;
}

template <class T> struct LocalB { std::vector<T> bx, by, bz; };

// gather the local nodal values of B_x, B_y, B_z of element e
template <class T> static LocalB<T> local_B(const Mesh& M, long e, const T* Bx, const T* By, const T* Bz) {
  long ex = e % M.nx, ey = e / M.nx;
  int a = M.m + 2, b = M.m + 1;
  LocalB<T> L;
  L.bx.resize(a * b); L.by.resize(a * b); L.bz.resize(b * b);
  for (int j = 0; j < b; ++j)
    for (int i = 0; i < a; ++i) L.bx[j * a + i] = Bx[gid(M, ex, ey, i, j)];
  for (int j = 0; j < a; ++j)
    for (int i = 0; i < b; ++i) L.by[j * b + i] = By[gid(M, ex, ey, i, j)];
  for (int j = 0; j < b; ++j)
    for (int i = 0; i < b; ++i) L.bz[j * b + i] = Bz[gid(M, ex, ey, i, j)];
  return L;
}

// Lumped auxiliary-product weights of element K for its local aux nodes
// (eq. quad-hcurl-element in physical components, eq. quad-cg-element).
static double wNx(const Mesh& M, int i, int j) { return M.J * M.og[i] * M.ow[j]; }
static double wNy(const Mesh& M, int i, int j) { return M.J * M.ow[i] * M.og[j]; }
static double wW(const Mesh& M, int i, int j) { return M.J * M.ow[i] * M.ow[j]; }

template <class T> struct Aux { std::vector<T> Jx, Jy, Jz, Ex, Ey, Ez; };

// Current reconstruction, eq. mag-current-proj: (J, chi)_A = (B, curl chi)_B with the
// exact B product (reading R17) and the lumped A product, gathered at shared nodes.
template <class T> static void reconstruct_J(const Mesh& M, const T* Bx, const T* By, const T* Bz,
                                             T* Jx, T* Jy, T* Jz) {
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  const int a = M.m + 2, b = M.m + 1;
  std::vector<T> lx(G, T(0.0)), ly(G, T(0.0)), lz(G, T(0.0));
  std::vector<double> mx(G, 0.0), my(G, 0.0), mz(G, 0.0);
  std::vector<T> locx((size_t)M.K * b * a), locy((size_t)M.K * a * b), locz((size_t)M.K * a * a);
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    LocalB<T> L = local_B(M, e, Bx, By, Bz);
    // W part: int_K B_x d_y phi_a - B_y d_x phi_a, (m+2)-point Gauss per direction
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) {
        T s = T(0.0);
        for (int qy = 0; qy < a; ++qy)
          for (int qx = 0; qx < a; ++qx) {
            double X = M.zq[qx], Y = M.zq[qy], wq = M.J * M.oq[qx] * M.oq[qy];
            T bxv = eval_tensor(M.xw, M.zg, L.bx.data(), X, Y, 0, 0);
            T byv = eval_tensor(M.zg, M.xw, L.by.data(), X, Y, 0, 0);
            double dyphi = lag(M.xw, i, X) * dlag(M.xw, j, Y) * (2.0 / M.hy);
            double dxphi = dlag(M.xw, i, X) * lag(M.xw, j, Y) * (2.0 / M.hx);
            s += wq * (bxv * dyphi - byv * dxphi);
          }
        locz[(size_t)e * a * a + j * a + i] = s;
      }
    // N part: int_K B_z (-d_y psi) for x-components, int_K B_z d_x psi for y-components,
    // (m+1)-point Gauss per direction (exact for the Q^m block)
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) {
        T s = T(0.0);
        for (int qy = 0; qy < b; ++qy)
          for (int qx = 0; qx < b; ++qx) {
            double X = M.zg[qx], Y = M.zg[qy], wq = M.J * M.og[qx] * M.og[qy];
            T bzv = eval_tensor(M.xv, M.xv, L.bz.data(), X, Y, 0, 0);
            s += wq * bzv * (-lag(M.zg, i, X) * dlag(M.xw, j, Y) * (2.0 / M.hy));
          }
        locx[(size_t)e * b * a + j * b + i] = s;
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) {
        T s = T(0.0);
        for (int qy = 0; qy < b; ++qy)
          for (int qx = 0; qx < b; ++qx) {
            double X = M.zg[qx], Y = M.zg[qy], wq = M.J * M.og[qx] * M.og[qy];
            T bzv = eval_tensor(M.xv, M.xv, L.bz.data(), X, Y, 0, 0);
            s += wq * bzv * (dlag(M.xw, i, X) * (2.0 / M.hx) * lag(M.zg, j, Y));
          }
        locy[(size_t)e * a * b + j * a + i] = s;
      }
  }
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) {
        long g = gid(M, ex, ey, i, j);
        lz[g] += locz[(size_t)e * a * a + j * a + i]; mz[g] += wW(M, i, j);
      }
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) {
        long g = gid(M, ex, ey, i, j);
        lx[g] += locx[(size_t)e * b * a + j * b + i]; mx[g] += wNx(M, i, j);
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) {
        long g = gid(M, ex, ey, i, j);
        ly[g] += locy[(size_t)e * a * b + j * a + i]; my[g] += wNy(M, i, j);
      }
  }
  for (long g = 0; g < G; ++g) { Jx[g] = lx[g] / mx[g]; Jy[g] = ly[g] / my[g]; Jz[g] = lz[g] / mz[g]; }
}

// J of element e evaluated at its GLL_p node (i,j): (Jx, Jy, Jz)
template <class T> static void J_at_gll(const Mesh& M, long e, const T* Jx, const T* Jy, const T* Jz,
                                        int i, int j, T* out) {
  long ex = e % M.nx, ey = e / M.nx;
  const int a = M.m + 2, b = M.m + 1;
  std::vector<T> vx(b * a), vy(a * b), vz(a * a);
  for (int jj = 0; jj < a; ++jj)
    for (int ii = 0; ii < b; ++ii) vx[jj * b + ii] = Jx[gid(M, ex, ey, ii, jj)];
  for (int jj = 0; jj < b; ++jj)
    for (int ii = 0; ii < a; ++ii) vy[jj * a + ii] = Jy[gid(M, ex, ey, ii, jj)];
  for (int jj = 0; jj < a; ++jj)
    for (int ii = 0; ii < a; ++ii) vz[jj * a + ii] = Jz[gid(M, ex, ey, ii, jj)];
  double X = M.xi[i], Y = M.xi[j];
  out[0] = eval_tensor(M.zg, M.xw, vx.data(), X, Y, 0, 0);
  out[1] = eval_tensor(M.xw, M.zg, vy.data(), X, Y, 0, 0);
  out[2] = eval_tensor(M.xw, M.xw, vz.data(), X, Y, 0, 0);
}

// u of element e at reference point (X,Y), interpolated from its GLL_p nodes
template <class T> static void u_at(const Mesh& M, long e, const T* u, double X, double Y, T* out) {
  for (int d = 0; d < 3; ++d) out[d] = eval_tensor(M.xi, M.xi, u + ((long)d * M.K + e) * M.nn, X, Y, 0, 0);
}
template <class T> static void B_at(const Mesh& M, const LocalB<T>& L, double X, double Y, T* out) {
  out[0] = eval_tensor(M.xw, M.zg, L.bx.data(), X, Y, 0, 0);
  out[1] = eval_tensor(M.zg, M.xw, L.by.data(), X, Y, 0, 0);
  out[2] = eval_tensor(M.xv, M.xv, L.bz.data(), X, Y, 0, 0);
}

// Electric-field reconstruction, eq. mag-electric-proj, with the ideal term evaluated
// from each element's own traces (reading R16) and the resistive term by the
// degree-p GLL rule.
template <class T> static void reconstruct_E(const Mesh& M, const T* u, const T* Bx, const T* By, const T* Bz,
                                             const T* Jx, const T* Jy, const T* Jz, const double* eta,
                                             T* Ex, T* Ey, T* Ez) {
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  const int a = M.m + 2, b = M.m + 1;
  std::vector<T> lx(G, T(0.0)), ly(G, T(0.0)), lz(G, T(0.0));
  std::vector<double> mx(G, 0.0), my(G, 0.0), mz(G, 0.0);
  std::vector<T> locx((size_t)M.K * b * a), locy((size_t)M.K * a * b), locz((size_t)M.K * a * a);
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    LocalB<T> L = local_B(M, e, Bx, By, Bz);
    double et = eta ? eta[e] : 0.0;
    std::vector<T> Jq((size_t)M.nn * 3);
    if (et != 0.0)
      for (int j = 0; j < M.np; ++j)
        for (int i = 0; i < M.np; ++i) J_at_gll(M, e, Jx, Jy, Jz, i, j, &Jq[(j * M.np + i) * 3]);
    auto node_load = [&](int comp, double X, double Y, double w, const std::vector<double>& nxs,
                         const std::vector<double>& nys, int ii, int jj) {
      T uu[3], BB[3];
      u_at(M, e, u, X, Y, uu);
      B_at(M, L, X, Y, BB);
      T cr = comp == 0 ? -(uu[1] * BB[2] - uu[2] * BB[1])
           : comp == 1 ? -(uu[2] * BB[0] - uu[0] * BB[2])
                       : -(uu[0] * BB[1] - uu[1] * BB[0]);
      T s = w * cr;
      if (et != 0.0) {
        for (int j = 0; j < M.np; ++j)
          for (int i = 0; i < M.np; ++i) {
            double phi = lag(nxs, ii, M.xi[i]) * lag(nys, jj, M.xi[j]);
            s += et * (M.J * M.om[i] * M.om[j]) * Jq[(j * M.np + i) * 3 + comp] * phi;
          }
      }
      return s;
    };
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i)
        locx[(size_t)e * b * a + j * b + i] = node_load(0, M.zg[i], M.xw[j], wNx(M, i, j), M.zg, M.xw, i, j);
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i)
        locy[(size_t)e * a * b + j * a + i] = node_load(1, M.xw[i], M.zg[j], wNy(M, i, j), M.xw, M.zg, i, j);
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i)
        locz[(size_t)e * a * a + j * a + i] = node_load(2, M.xw[i], M.xw[j], wW(M, i, j), M.xw, M.xw, i, j);
  }
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) {
        long g = gid(M, ex, ey, i, j);
        lx[g] += locx[(size_t)e * b * a + j * b + i]; mx[g] += wNx(M, i, j);
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) {
        long g = gid(M, ex, ey, i, j);
        ly[g] += locy[(size_t)e * a * b + j * a + i]; my[g] += wNy(M, i, j);
      }
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) {
        long g = gid(M, ex, ey, i, j);
        lz[g] += locz[(size_t)e * a * a + j * a + i]; mz[g] += wW(M, i, j);
      }
  }
  for (long g = 0; g < G; ++g) { Ex[g] = lx[g] / mx[g]; Ey[g] = ly[g] / my[g]; Ez[g] = lz[g] / mz[g]; }
}

// L_M: mass-inverted magnetic operator (eq. magnetic-dae with J, E eliminated).
// Outputs de [K][nn], du [3][K][nn], dBx, dBy, dBz grids.  Optional J, E outputs.
template <class T>
static void rhs_magnetic_t(const Mesh& M, const double* rho, const T* u, const T* Bx, const T* By,
                           const T* Bz, const double* eta, T* de, T* du, T* dBx, T* dBy, T* dBz,
                           T* Jout /*6 grids or null*/) {
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  const int a = M.m + 2, b = M.m + 1;
  std::vector<T> Jx(G), Jy(G), Jz(G), Ex(G), Ey(G), Ez(G);
  reconstruct_J(M, Bx, By, Bz, Jx.data(), Jy.data(), Jz.data());
  reconstruct_E(M, u, Bx, By, Bz, Jx.data(), Jy.data(), Jz.data(), eta, Ex.data(), Ey.data(), Ez.data());
  if (Jout) {
    for (long g = 0; g < G; ++g) {
      Jout[g] = Jx[g]; Jout[G + g] = Jy[g]; Jout[2 * G + g] = Jz[g];
      Jout[3 * G + g] = Ex[g]; Jout[4 * G + g] = Ey[g]; Jout[5 * G + g] = Ez[g];
    }
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    std::vector<T> vEz(a * a), vEx(b * a), vEy(a * b);
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) vEz[j * a + i] = Ez[gid(M, ex, ey, i, j)];
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) vEx[j * b + i] = Ex[gid(M, ex, ey, i, j)];
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) vEy[j * a + i] = Ey[gid(M, ex, ey, i, j)];
    // strong curl (section "Semidiscrete differential-algebraic formulation");
    // each shared B_x / B_y node is written by the element that owns local index 0..m
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) {
        double X = M.xw[i], Y = M.zg[j];
        dBx[gid(M, ex, ey, i, j)] = -eval_tensor(M.xw, M.xw, vEz.data(), X, Y, 0, 1) * (2.0 / M.hy);
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) {
        double X = M.zg[i], Y = M.xw[j];
        dBy[gid(M, ex, ey, i, j)] = eval_tensor(M.xw, M.xw, vEz.data(), X, Y, 1, 0) * (2.0 / M.hx);
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) {
        double X = M.xv[i], Y = M.xv[j];
        T dxEy = eval_tensor(M.xw, M.zg, vEy.data(), X, Y, 1, 0) * (2.0 / M.hx);
        T dyEx = eval_tensor(M.zg, M.xw, vEx.data(), X, Y, 0, 1) * (2.0 / M.hy);
        dBz[gid(M, ex, ey, i, j)] = -(dxEy - dyEx);
      }
    // Lorentz load (algebraic transpose of the coupling form) and Ohmic heating
    LocalB<T> L = local_B(M, e, Bx, By, Bz);
    std::vector<T> fu((size_t)3 * M.nn, T(0.0));
    auto add_node = [&](double X, double Y, double w, const T* f) {
      for (int q = 0; q < M.nn; ++q) {
        double I = lag(M.xi, q % M.np, X) * lag(M.xi, q / M.np, Y);
        for (int d = 0; d < 3; ++d) fu[(size_t)d * M.nn + q] += w * I * f[d];
      }
    };
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) {  // N_x nodes: f = (0, -B_z J_x, B_y J_x)
        double X = M.zg[i], Y = M.xw[j];
        T BB[3]; B_at(M, L, X, Y, BB);
        T J = Jx[gid(M, ex, ey, i, j)];
        T f[3] = {T(0.0), -BB[2] * J, BB[1] * J};
        add_node(X, Y, wNx(M, i, j), f);
      }
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) {  // N_y nodes: f = (B_z J_y, 0, -B_x J_y)
        double X = M.xw[i], Y = M.zg[j];
        T BB[3]; B_at(M, L, X, Y, BB);
        T J = Jy[gid(M, ex, ey, i, j)];
        T f[3] = {BB[2] * J, T(0.0), -BB[0] * J};
        add_node(X, Y, wNy(M, i, j), f);
      }
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) {  // W nodes: f = (-B_y J_z, B_x J_z, 0)
        double X = M.xw[i], Y = M.xw[j];
        T BB[3]; B_at(M, L, X, Y, BB);
        T J = Jz[gid(M, ex, ey, i, j)];
        T f[3] = {-BB[1] * J, BB[0] * J, T(0.0)};
        add_node(X, Y, wW(M, i, j), f);
      }
    double et = eta ? eta[e] : 0.0;
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) {
        int q = j * M.np + i;
        double rq = rho[(long)e * M.nn + q], Mq = M.J * M.om[i] * M.om[j];
        for (int d = 0; d < 3; ++d) du[((long)d * M.K + e) * M.nn + q] = fu[(size_t)d * M.nn + q] / (rq * Mq);
        T Jv[3] = {T(0.0), T(0.0), T(0.0)};
        if (et != 0.0) J_at_gll(M, e, Jx.data(), Jy.data(), Jz.data(), i, j, Jv);
        de[(long)e * M.nn + q] = et * (Jv[0] * Jv[0] + Jv[1] * Jv[1] + Jv[2] * Jv[2]) / rq;
      }
  }
}

// B at the GLL_p nodes of element e
static void B_at_gll(const Mesh& M, long e, const double* Bx, const double* By, const double* Bz, double* out /*[nn][3]*/) {
  LocalB<double> L = local_B(M, e, Bx, By, Bz);
  for (int j = 0; j < M.np; ++j)
    for (int i = 0; i < M.np; ++i) B_at(M, L, M.xi[i], M.xi[j], &out[(j * M.np + i) * 3]);
}

// Global amplitude Delta_Omega of a magnetic component over its own DOF nodes, with
// its mean taken as the exact integral over Omega (reading R18).  comp 0,1,2 = x,y,z.
static void B_global_amp(const Mesh& M, const double* Bx, const double* By, const double* Bz, int comp,
                         double* dOm, int* cflag) {
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  const double* f = comp == 0 ? Bx : comp == 1 ? By : Bz;
  double integ = 0.0;
  const int nq = M.m + 2;
  for (long e = 0; e < M.K; ++e) {
    if (!in_box(M, e)) continue;
    LocalB<double> L = local_B(M, e, Bx, By, Bz);
    for (int qy = 0; qy < nq; ++qy)
      for (int qx = 0; qx < nq; ++qx) {
        double BB[3]; B_at(M, L, M.zq[qx], M.zq[qy], BB);
        integ += M.J * M.oq[qx] * M.oq[qy] * BB[comp];
      }
  }
  double mean = integ / ((double)M.bx * M.by * M.hx * M.hy), d = 0.0, amax = 0.0, vmin = f[0], vmax = f[0];
  // the box's DOFs: grid columns (rows) up to bx (by) (m+1) positions, and the wall position itself
  // where the component's nodes in that direction are the shared GLL_{m+1} nodes (B_x in x, B_y in y)
  const long NXg = (long)M.nx * M.M1, lim_x = (long)M.bx * M.M1 + ((M.walls & 1) && comp == 0 ? 1 : 0),
             lim_y = (long)M.by * M.M1 + ((M.walls & 2) && comp == 1 ? 1 : 0);
  for (long g = 0; g < G; ++g) {
    if (g % NXg >= lim_x || g / NXg >= lim_y) continue;
    d = std::max(d, std::fabs(f[g] - mean)); amax = std::max(amax, std::fabs(f[g]));
    vmin = std::min(vmin, f[g]); vmax = std::max(vmax, f[g]);
  }
  *dOm = d;
  // roundoff-level variation: the DOF values agree to 2^10 ulps of the component's size (exact test)
  *cflag = vmax - vmin <= 1024.0 * EPS * amax ? 1 : 0;
}

// Artificial-resistivity coefficient eta_K (eq. magnetic-ar-sensor, eq. magnetic-ar-coefficient).
static void ar_eta(const Mesh& M, const Opts& o, const double* rho, const double* u, const double* Bx,
                   const double* By, const double* Bz, double* eta) {
  double dOm[3]; int cf[3];
  for (int c = 0; c < 3; ++c) B_global_amp(M, Bx, By, Bz, c, &dOm[c], &cf[c]);
  const int nq = M.m + 2;
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    double Rdir[2], adir[2];
    for (int dir = 0; dir < 2; ++dir) {
      // tangential components to faces normal to x: {y, z}; normal to y: {x, z}
      int t0 = dir == 0 ? 1 : 0, t1 = 2;
      double DB = std::max(cf[t0] ? 0.0 : dOm[t0], cf[t1] ? 0.0 : dOm[t1]);
      double sig = 0.0;
      if (DB > 0.0) {
        long em = dir == 0 ? elem(M, ex - 1, ey) : elem(M, ex, ey - 1);
        long ep = dir == 0 ? elem(M, ex + 1, ey) : elem(M, ex, ey + 1);
        LocalB<double> L = local_B(M, e, Bx, By, Bz), Lm = local_B(M, em, Bx, By, Bz), Lp = local_B(M, ep, Bx, By, Bz);
        for (int tc : {t0, t1}) {
          if (cf[tc]) continue;
          double sm = 0.0, sp = 0.0;
          for (int k = 0; k < nq; ++k) {
            double s = M.zq[k];
            double X0 = dir == 0 ? -1.0 : s, Y0 = dir == 0 ? s : -1.0;
            double X1 = dir == 0 ? 1.0 : s, Y1 = dir == 0 ? s : 1.0;
            double own0[3], own1[3], nb0[3], nb1[3];
            B_at(M, L, X0, Y0, own0); B_at(M, L, X1, Y1, own1);
            B_at(M, Lm, X1, Y1, nb0); B_at(M, Lp, X0, Y0, nb1);
            double jm = own0[tc] - nb0[tc], jp = nb1[tc] - own1[tc];
            sm += 0.5 * M.oq[k] * jm * jm;
            sp += 0.5 * M.oq[k] * jp * jp;
          }
          sig = std::max(sig, (std::sqrt(sm) + std::sqrt(sp)) / (2.0 * DB));
        }
      }
      Rdir[dir] = std::min(o.Cs * sig, 1.0);
    }
    std::vector<double> Bq((size_t)M.nn * 3);
    B_at_gll(M, e, Bx, By, Bz, Bq.data());
    adir[0] = adir[1] = 0.0;
    for (int q = 0; q < M.nn; ++q) {
      double bb = std::sqrt(Bq[q * 3] * Bq[q * 3] + Bq[q * 3 + 1] * Bq[q * 3 + 1] + Bq[q * 3 + 2] * Bq[q * 3 + 2]);
      double va = bb / std::sqrt(rho[(long)e * M.nn + q]);
      adir[0] = std::max(adir[0], std::fabs(u[((long)0 * M.K + e) * M.nn + q]) + va);
      adir[1] = std::max(adir[1], std::fabs(u[((long)1 * M.K + e) * M.nn + q]) + va);
    }
    double v0 = M.hx / (2.0 * M.p + 1.0) * adir[0] * Rdir[0];
    double v1 = M.hy / (2.0 * M.p + 1.0) * adir[1] * Rdir[1];
    eta[e] = o.Ceta * std::max(v0, v1);
  }
}

// Velocity OE (eq. magnetic-oe-sensor .. eq. magnetic-oe-map) on a raw stage (u, e, B).
static void velocity_oe(const Mesh& M, const Opts& o, double tau, const double* rho, double* u, double* en,
                        const double* Bx, const double* By, const double* Bz, double* Dout) {
  const int nn = M.nn;
  std::vector<LineStats> S(3);
  for (int d = 0; d < 3; ++d) S[d] = line_stats(M, u + (long)d * M.K * nn);
  std::vector<double> uin(u, u + 3 * M.K * nn);
#pragma omp parallel for schedule(dynamic, 16)
  for (long e = 0; e < M.K; ++e) {
    const double* fields[3] = {uin.data(), uin.data() + M.K * nn, uin.data() + 2 * M.K * nn};
    std::vector<double> sig;
    oe_sensor(M, e, 3, fields, S, sig);
    std::vector<double> Bq((size_t)nn * 3);
    B_at_gll(M, e, Bx, By, Bz, Bq.data());
    double amax[2] = {0.0, 0.0};
    for (int q = 0; q < nn; ++q) {
      double bb = std::sqrt(Bq[q * 3] * Bq[q * 3] + Bq[q * 3 + 1] * Bq[q * 3 + 1] + Bq[q * 3 + 2] * Bq[q * 3 + 2]);
      double va = bb / std::sqrt(rho[(long)e * nn + q]);
      amax[0] = std::max(amax[0], std::fabs(fields[0][(long)e * nn + q]) + va);
      amax[1] = std::max(amax[1], std::fabs(fields[1][(long)e * nn + q]) + va);
    }
    double lam[2] = {(2.0 * M.p + 1.0) / M.hx * amax[0], (2.0 * M.p + 1.0) / M.hy * amax[1]};
    std::vector<double> D(M.np, 1.0);
    for (int l = 1; l <= M.p; ++l) {
      double Th = 0.0;
      for (int dir = 0; dir < 2; ++dir) {
        double s = 0.0;
        for (int r = 0; r <= l; ++r) s += sig[dir * M.np + r];
        Th += lam[dir] * s;
      }
      D[l] = std::exp(-o.sM * tau * Th);
    }
    if (Dout) for (int l = 0; l <= M.p; ++l) Dout[e * M.np + l] = D[l];
    std::vector<double> Wq(nn);
    for (int j = 0; j < M.np; ++j)
      for (int i = 0; i < M.np; ++i) Wq[j * M.np + i] = M.J * M.om[i] * M.om[j] * rho[(long)e * nn + j * M.np + i];
    std::vector<double> heat(nn, 0.0);
    for (int d = 0; d < 3; ++d) {
      std::vector<double> P;
      projections(M, fields[d] + (long)e * nn, Wq.data(), P);
      for (int q = 0; q < nn; ++q) {
        double v = P[q];
        for (int l = 1; l <= M.p; ++l) {
          double wl = P[(size_t)l * nn + q] - P[(size_t)(l - 1) * nn + q];
          v += D[l] * wl;
          heat[q] += 0.5 * (1.0 - D[l] * D[l]) * wl * wl;
        }
        u[((long)d * M.K + e) * nn + q] = v;
      }
    }
    for (int q = 0; q < nn; ++q) en[(long)e * nn + q] += heat[q];
  }
}

// Magnetic-velocity substep (Algorithm "Magnetic-velocity substep", eq. magnetic-ssprk33).
static void magnetic_substep(const Mesh& M, const Opts& o, const double* rho, double* en, double* u, double* Bx,
                             double* By, double* Bz, double tau, Report* rep) {
  const long nn = M.K * M.nn, G = (long)M.nx * M.ny * M.M1 * M.M1;
  std::vector<double> eta(M.K, 0.0);
  if (o.ar && o.Ceta > 0.0) ar_eta(M, o, rho, u, Bx, By, Bz, eta.data());
  if (rep) { double mx = 0.0; for (long e = 0; e < M.K; ++e) mx = std::max(mx, eta[e]); rep->eta_max = mx; }
  // Y = (e, u, B) packed as [e | u | Bx | By | Bz]
  const long n = nn + 3 * nn + 3 * G;
  std::vector<double> Yn(n), Y1(n), Y2(n), Ys(n), L(n);
  auto pack = [&](std::vector<double>& Y, const double* e_, const double* u_, const double* bx, const double* by,
                  const double* bz) {
    std::memcpy(&Y[0], e_, nn * sizeof(double)); std::memcpy(&Y[nn], u_, 3 * nn * sizeof(double));
    std::memcpy(&Y[4 * nn], bx, G * sizeof(double)); std::memcpy(&Y[4 * nn + G], by, G * sizeof(double));
    std::memcpy(&Y[4 * nn + 2 * G], bz, G * sizeof(double));
  };
  pack(Yn, en, u, Bx, By, Bz);
  auto rhs = [&](const std::vector<double>& Y, std::vector<double>& out) {
    rhs_magnetic_t<double>(M, rho, &Y[nn], &Y[4 * nn], &Y[4 * nn + G], &Y[4 * nn + 2 * G],
                           (o.ar && o.Ceta > 0.0) ? eta.data() : nullptr, &out[0], &out[nn], &out[4 * nn],
                           &out[4 * nn + G], &out[4 * nn + 2 * G], nullptr);
  };
  auto stage_map = [&](std::vector<double>& Y) {
    if (o.oe_mag) velocity_oe(M, o, tau, rho, &Y[nn], &Y[0], &Y[4 * nn], &Y[4 * nn + G], &Y[4 * nn + 2 * G], nullptr);
  };
  rhs(Yn, L);
  for (long q = 0; q < n; ++q) Ys[q] = Yn[q] + tau * L[q];
  stage_map(Ys); Y1 = Ys;
  rhs(Y1, L);
  for (long q = 0; q < n; ++q) Ys[q] = 0.75 * Yn[q] + 0.25 * (Y1[q] + tau * L[q]);
  stage_map(Ys); Y2 = Ys;
  rhs(Y2, L);
  for (long q = 0; q < n; ++q) Ys[q] = (1.0 / 3.0) * Yn[q] + (2.0 / 3.0) * (Y2[q] + tau * L[q]);
  stage_map(Ys);
  std::memcpy(en, &Ys[0], nn * sizeof(double)); std::memcpy(u, &Ys[nn], 3 * nn * sizeof(double));
  std::memcpy(Bx, &Ys[4 * nn], G * sizeof(double)); std::memcpy(By, &Ys[4 * nn + G], G * sizeof(double));
  std::memcpy(Bz, &Ys[4 * nn + 2 * G], G * sizeof(double));
}

// Nodal variable exchange (section "Local variable exchange").
static void to_primitive(const Mesh& M, const double* U, double* rho, double* en, double* u) {
  const long nn = M.K * M.nn;
  for (long q = 0; q < nn; ++q) {
    double r = U[q];
    double ux = U[nn + q] / r, uy = U[2 * nn + q] / r, uz = U[3 * nn + q] / r;
    rho[q] = r; u[q] = ux; u[nn + q] = uy; u[2 * nn + q] = uz;
    en[q] = (U[4 * nn + q] - 0.5 * r * (ux * ux + uy * uy + uz * uz)) / r;
  }
}
static void to_conservative(const Mesh& M, const double* rho, const double* en, const double* u, double* U) {
  const long nn = M.K * M.nn;
  for (long q = 0; q < nn; ++q) {
    double r = rho[q], ux = u[q], uy = u[nn + q], uz = u[2 * nn + q];
    U[q] = r; U[nn + q] = r * ux; U[2 * nn + q] = r * uy; U[3 * nn + q] = r * uz;
    U[4 * nn + q] = r * en[q] + 0.5 * r * (ux * ux + uy * uy + uz * uz);
  }
}

// ---------------------------------------------------------------------------
// extern "C" entry points (host pointers; see oracle/__init__.py)
// ---------------------------------------------------------------------------
extern "C" {

int or_tables(int kind, int r, double* x, double* w) {
  std::vector<double> X, W;
  if (kind == 0) gll_rule(r, X, W); else gauss_rule(r + 1, X, W);
  for (size_t k = 0; k < X.size(); ++k) { x[k] = X[k]; w[k] = W[k]; }
  return 0;
}

int or_diff_matrix(int r, double* D) {
  std::vector<double> X, W; gll_rule(r, X, W);
  for (int i = 0; i <= r; ++i)
    for (int j = 0; j <= r; ++j) D[i * (r + 1) + j] = dlag(X, j, X[i]);
  return 0;
}

int or_ec_flux(const double* UL, const double* UR, int d, double gamma, double* F) {
  St<double> L{UL[0], UL[1], UL[2], UL[3], UL[4]}, R{UR[0], UR[1], UR[2], UR[3], UR[4]};
  ec_flux(L, R, d, gamma, F);
  return 0;
}
int or_phys_flux(const double* U, int d, double gamma, double* F) {
  St<double> s{U[0], U[1], U[2], U[3], U[4]};
  phys_flux(s, d, gamma, F);
  return 0;
}
int or_llf_flux(const double* UL, const double* UR, int d, double gamma, double* F) {
  St<double> L{UL[0], UL[1], UL[2], UL[3], UL[4]}, R{UR[0], UR[1], UR[2], UR[3], UR[4]};
  llf_flux(L, R, d, gamma, F);
  return 0;
}
double or_logmean(double a, double b) { return logmean(a, b); }

int or_rhs_hydro(const int* im, const double* dm, int iface_flux, const double* U, double* dU) {
  Mesh M = make_mesh(im, dm);
  rhs_hydro_t<double>(M, iface_flux, U, dU);
  return 0;
}

// forward-mode complex-step JVP of L_E: dU = Im(L_E(U + i h V))/h
int or_rhs_hydro_jvp(const int* im, const double* dm, int iface_flux, const double* U, const double* V, double* JV) {
  Mesh M = make_mesh(im, dm);
  const long n = 5 * M.K * M.nn;
  const double h = 1e-30;
  std::vector<cplx> Uc(n), dc(n);
  for (long q = 0; q < n; ++q) Uc[q] = cplx(U[q], h * V[q]);
  rhs_hydro_t<cplx>(M, iface_flux, Uc.data(), dc.data());
  for (long q = 0; q < n; ++q) JV[q] = dc[q].imag() / h;
  return 0;
}

int or_hydro_stage_map(const int* im, const double* dm, const int* io, const double* dop, double tau, double* U,
                       uint8_t* flags, int64_t* counts, double* Dout) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  int64_t c[3] = {0, 0, 0};
  hydro_stage_map(M, o, tau, U, flags, c, Dout);
  if (counts) { counts[0] = c[0]; counts[1] = c[1]; counts[2] = c[2]; }
  return 0;
}

int or_averages_admissible(const int* im, const double* dm, const double* U) {
  Mesh M = make_mesh(im, dm);
  return averages_admissible(M, U) ? 1 : 0;
}

int or_hydro_substep(const int* im, const double* dm, const int* io, const double* dop, double* U, double tau,
                     Report* rep, uint8_t* flags, int32_t* log, int log_cap) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  std::memset(rep, 0, sizeof(Report));
  rep->dt = tau;
  if (!state_admissible(M, U)) { rep->status = 2; return 2; }
  std::vector<double> save(U, U + 5 * M.K * M.nn);
  int s = hydro_substep_rec(M, o, U, tau, 0, rep, flags, log, log_cap);
  if (s) std::memcpy(U, save.data(), save.size() * sizeof(double));
  rep->status = s;
  return s;
}

int or_reconstruct_JE(const int* im, const double* dm, const double* u, const double* Bx, const double* By,
                      const double* Bz, const double* eta, double* out6) {
  Mesh M = make_mesh(im, dm);
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  reconstruct_J<double>(M, Bx, By, Bz, out6, out6 + G, out6 + 2 * G);
  reconstruct_E<double>(M, u, Bx, By, Bz, out6, out6 + G, out6 + 2 * G, eta, out6 + 3 * G, out6 + 4 * G, out6 + 5 * G);
  return 0;
}

int or_rhs_magnetic(const int* im, const double* dm, const double* rho, const double* u, const double* Bx,
                    const double* By, const double* Bz, const double* eta, double* de, double* du, double* dBx,
                    double* dBy, double* dBz) {
  Mesh M = make_mesh(im, dm);
  rhs_magnetic_t<double>(M, rho, u, Bx, By, Bz, eta, de, du, dBx, dBy, dBz, nullptr);
  return 0;
}

// complex-step JVP of L_M in the direction (Vu, VBx, VBy, VBz); rho and eta frozen
int or_rhs_magnetic_jvp(const int* im, const double* dm, const double* rho, const double* u, const double* Bx,
                        const double* By, const double* Bz, const double* eta, const double* Vu, const double* VBx,
                        const double* VBy, const double* VBz, double* de, double* du, double* dBx, double* dBy,
                        double* dBz) {
  Mesh M = make_mesh(im, dm);
  const long nn = M.K * M.nn, G = (long)M.nx * M.ny * M.M1 * M.M1;
  const double h = 1e-30;
  std::vector<cplx> uc(3 * nn), bx(G), by(G), bz(G), oe(nn), ou(3 * nn), ox(G), oy(G), oz(G);
  for (long q = 0; q < 3 * nn; ++q) uc[q] = cplx(u[q], h * Vu[q]);
  for (long g = 0; g < G; ++g) { bx[g] = cplx(Bx[g], h * VBx[g]); by[g] = cplx(By[g], h * VBy[g]); bz[g] = cplx(Bz[g], h * VBz[g]); }
  rhs_magnetic_t<cplx>(M, rho, uc.data(), bx.data(), by.data(), bz.data(), eta, oe.data(), ou.data(), ox.data(),
                       oy.data(), oz.data(), nullptr);
  for (long q = 0; q < nn; ++q) de[q] = oe[q].imag() / h;
  for (long q = 0; q < 3 * nn; ++q) du[q] = ou[q].imag() / h;
  for (long g = 0; g < G; ++g) { dBx[g] = ox[g].imag() / h; dBy[g] = oy[g].imag() / h; dBz[g] = oz[g].imag() / h; }
  return 0;
}

int or_ar_eta(const int* im, const double* dm, const int* io, const double* dop, const double* rho, const double* u,
              const double* Bx, const double* By, const double* Bz, double* eta) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  ar_eta(M, o, rho, u, Bx, By, Bz, eta);
  return 0;
}

int or_velocity_oe(const int* im, const double* dm, const int* io, const double* dop, double tau, const double* rho,
                   double* u, double* en, const double* Bx, const double* By, const double* Bz, double* Dout) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  velocity_oe(M, o, tau, rho, u, en, Bx, By, Bz, Dout);
  return 0;
}

int or_step_magnetic(const int* im, const double* dm, const int* io, const double* dop, const double* rho, double* en,
                     double* u, double* Bx, double* By, double* Bz, double tau, Report* rep) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  if (rep) { std::memset(rep, 0, sizeof(Report)); rep->dt = tau; }
  const long G = (long)M.nx * M.ny * M.M1 * M.M1;
  if (!primitive_admissible(M, rho, en, u) || !all_finite(Bx, G) || !all_finite(By, G) || !all_finite(Bz, G)) {
    if (rep) rep->status = 2;
    return 2;
  }
  magnetic_substep(M, o, rho, en, u, Bx, By, Bz, tau, rep);
  return 0;
}

int or_to_primitive(const int* im, const double* dm, const double* U, double* rho, double* en, double* u) {
  Mesh M = make_mesh(im, dm);
  to_primitive(M, U, rho, en, u);
  return 0;
}
int or_to_conservative(const int* im, const double* dm, const double* rho, const double* en, const double* u, double* U) {
  Mesh M = make_mesh(im, dm);
  to_conservative(M, rho, en, u, U);
  return 0;
}

// Strang step (Algorithm "Strang split MHD step", eq. strang-composition): the composition the paper
// states, H(dt/2) M(dt) H(dt/2) (strang_order 0), or the magnetic-outer one, M(dt/2) H(dt) M(dt/2)
// (strang_order 1), whose results reproduce the magnitudes of the paper's temporal self-convergence
// table (the stated composition gives the printed rates but Cauchy differences 4.6 to 9 times
// smaller).  The exchange of section "Local variable exchange" joins the maps.
int or_strang_step(const int* im, const double* dm, const int* io, const double* dop, double* U, double* Bx,
                   double* By, double* Bz, double dt, Report* rep, uint8_t* flags) {
  Mesh M = make_mesh(im, dm); Opts o = make_opts(io, dop);
  std::memset(rep, 0, sizeof(Report));
  rep->dt = dt;
  const long nn = M.K * M.nn, G = (long)M.nx * M.ny * M.M1 * M.M1;
  if (!state_admissible(M, U) || !all_finite(Bx, G) || !all_finite(By, G) || !all_finite(Bz, G)) {
    rep->status = 2;
    return 2;
  }
  std::vector<double> save(U, U + 5 * nn), sbx(Bx, Bx + G), sby(By, By + G), sbz(Bz, Bz + G);
  std::vector<double> rho(nn), en(nn), u(3 * nn);
  auto restore = [&]() {
    std::memcpy(U, save.data(), save.size() * sizeof(double));
    std::memcpy(Bx, sbx.data(), G * sizeof(double)); std::memcpy(By, sby.data(), G * sizeof(double));
    std::memcpy(Bz, sbz.data(), G * sizeof(double));
  };
  auto magnetic = [&](double tau, Report* rm) {
    to_primitive(M, U, rho.data(), en.data(), u.data());
    magnetic_substep(M, o, rho.data(), en.data(), u.data(), Bx, By, Bz, tau, rm);
    to_conservative(M, rho.data(), en.data(), u.data(), U);
  };
  Report r1, r2, rm;
  std::memset(&r1, 0, sizeof(r1)); std::memset(&r2, 0, sizeof(r2)); std::memset(&rm, 0, sizeof(rm));
  int s = 0;
  if (o.strang_order == 0) {
    s = hydro_substep_rec(M, o, U, 0.5 * dt, 0, &r1, flags, nullptr, 0);
    if (s) { restore(); rep->status = s; return s; }
    magnetic(dt, &rm);
    s = hydro_substep_rec(M, o, U, 0.5 * dt, 0, &r2, flags, nullptr, 0);
  } else {
    magnetic(0.5 * dt, &rm);
    s = hydro_substep_rec(M, o, U, dt, 0, &r1, flags, nullptr, 0);
    if (!s) magnetic(0.5 * dt, &rm);
  }
  if (s) restore();
  rep->attempted = r1.attempted + r2.attempted; rep->accepted = r1.accepted + r2.accepted;
  rep->max_depth = std::max(r1.max_depth, r2.max_depth);
  rep->n_rho = r1.n_rho + r2.n_rho; rep->n_p = r1.n_p + r2.n_p; rep->n_col = r1.n_col + r2.n_col;
  rep->eta_max = rm.eta_max; rep->status = s;
  return s;
}

// Exact magnetic energy-product (C, D)_B (eq. magnetic-inner-product) of two B fields.
double or_B_product(const int* im, const double* dm, const double* Cx, const double* Cy, const double* Cz,
                    const double* Dx, const double* Dy, const double* Dz) {
  Mesh M = make_mesh(im, dm);
  double s = 0.0;
  const int a = M.m + 2, b = M.m + 1;
  for (long e = 0; e < M.K; ++e) {
    LocalB<double> Lc = local_B(M, e, Cx, Cy, Cz), Ld = local_B(M, e, Dx, Dy, Dz);
    for (int qy = 0; qy < a; ++qy)
      for (int qx = 0; qx < a; ++qx) {
        double X = M.zq[qx], Y = M.zq[qy], w = M.J * M.oq[qx] * M.oq[qy];
        s += w * (eval_tensor(M.xw, M.zg, Lc.bx.data(), X, Y, 0, 0) * eval_tensor(M.xw, M.zg, Ld.bx.data(), X, Y, 0, 0) +
                  eval_tensor(M.zg, M.xw, Lc.by.data(), X, Y, 0, 0) * eval_tensor(M.zg, M.xw, Ld.by.data(), X, Y, 0, 0));
      }
    for (int qy = 0; qy < b; ++qy)
      for (int qx = 0; qx < b; ++qx) {
        double X = M.zg[qx], Y = M.zg[qy], w = M.J * M.og[qx] * M.og[qy];
        s += w * eval_tensor(M.xv, M.xv, Lc.bz.data(), X, Y, 0, 0) * eval_tensor(M.xv, M.xv, Ld.bz.data(), X, Y, 0, 0);
      }
  }
  return s;
}

// B_par = grad^perp A_h = (-d_y A, d_x A) for A_h in W^{m+1} given at its global nodes (helper for
// divergence-free initial data, section "Advected MHD vortex").
int or_B_from_potential(const int* im, const double* dm, const double* A, double* Bx, double* By) {
  Mesh M = make_mesh(im, dm);
  const int a = M.m + 2, b = M.m + 1;
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    std::vector<double> v(a * a);
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < a; ++i) v[j * a + i] = A[gid(M, ex, ey, i, j)];
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < b; ++i) {
        Bx[gid(M, ex, ey, i, j)] = -eval_tensor(M.xw, M.xw, v.data(), M.xw[i], M.zg[j], 0, 1) * (2.0 / M.hy);
        By[gid(M, ex, ey, i, j)] = eval_tensor(M.xw, M.xw, v.data(), M.zg[i], M.xw[j], 1, 0) * (2.0 / M.hx);
      }
  }
  return 0;
}

// ||div B_par||_{L2(Omega)} by (m+2)-point Gauss on each element.
double or_divB_L2(const int* im, const double* dm, const double* Bx, const double* By) {
  Mesh M = make_mesh(im, dm);
  const int a = M.m + 2, b = M.m + 1;
  double s = 0.0;
  for (long e = 0; e < M.K; ++e) {
    long ex = e % M.nx, ey = e / M.nx;
    std::vector<double> vx(a * b), vy(b * a);
    for (int j = 0; j < b; ++j)
      for (int i = 0; i < a; ++i) vx[j * a + i] = Bx[gid(M, ex, ey, i, j)];
    for (int j = 0; j < a; ++j)
      for (int i = 0; i < b; ++i) vy[j * b + i] = By[gid(M, ex, ey, i, j)];
    for (int qy = 0; qy < a; ++qy)
      for (int qx = 0; qx < a; ++qx) {
        double X = M.zq[qx], Y = M.zq[qy];
        double dv = eval_tensor(M.xw, M.zg, vx.data(), X, Y, 1, 0) * (2.0 / M.hx) +
                    eval_tensor(M.zg, M.xw, vy.data(), X, Y, 0, 1) * (2.0 / M.hy);
        s += M.J * M.oq[qx] * M.oq[qy] * dv * dv;
      }
  }
  return std::sqrt(s);
}

// evaluate B (3 comps) of element e at reference points (used by error norms in tests)
int or_eval_B(const int* im, const double* dm, const double* Bx, const double* By, const double* Bz, long e, int npts,
              const double* X, const double* Y, double* out) {
  Mesh M = make_mesh(im, dm);
  LocalB<double> L = local_B(M, e, Bx, By, Bz);
  for (int k = 0; k < npts; ++k) B_at(M, L, X[k], Y[k], out + 3 * k);
  return 0;
}

// Physical coordinates of the nodes of one node set (space 0: GLL_p element nodes [K][p+1][p+1];
// 1: B_x grid; 2: B_y grid; 3: B_z grid; 4: E_z/J_z grid (W); 5: E_x/J_x grid (N_x); 6: E_y/J_y
// grid (N_y)).  A grid node with global index (gy, gx) belongs to element (gx / (m+1), gy / (m+1))
// as its local node (gx mod (m+1), gy mod (m+1)); a shared GLL_{m+1} node is its first local node.
int or_node_coords(const int* im, const double* dm, int space, double* x, double* y) {
  Mesh M = make_mesh(im, dm);
  if (space == 0) {
    for (long e = 0; e < M.K; ++e) {
      const long ex = e % M.nx, ey = e / M.nx;
      for (int j = 0; j < M.np; ++j)
        for (int i = 0; i < M.np; ++i) {
          x[nid(M, 0, e, i, j)] = M.x0 + M.hx * ex + 0.5 * (M.xi[i] + 1.0) * M.hx;
          y[nid(M, 0, e, i, j)] = M.y0 + M.hy * ey + 0.5 * (M.xi[j] + 1.0) * M.hy;
        }
    }
    return 0;
  }
  if (space < 1 || space > 6) return -1;
  // 1D node sets per direction: GLL_{m+1} (first m+1 nodes), Gauss_m, GLL_m
  const std::vector<double>* sx;
  const std::vector<double>* sy;
  switch (space) {
    case 1: sx = &M.xw; sy = &M.zg; break;   // B_x: GLL_{m+1} x Gauss_m
    case 2: sx = &M.zg; sy = &M.xw; break;   // B_y: Gauss_m x GLL_{m+1}
    case 3: sx = &M.xv; sy = &M.xv; break;   // B_z: GLL_m x GLL_m
    case 4: sx = &M.xw; sy = &M.xw; break;   // W: GLL_{m+1} x GLL_{m+1}
    case 5: sx = &M.zg; sy = &M.xw; break;   // N_x: Gauss_m x GLL_{m+1}
    default: sx = &M.xw; sy = &M.zg; break;  // N_y: GLL_{m+1} x Gauss_m
  }
  for (long ey = 0; ey < M.ny; ++ey)
    for (long ex = 0; ex < M.nx; ++ex)
      for (int j = 0; j < M.M1; ++j)
        for (int i = 0; i < M.M1; ++i) {
          const long g = gid(M, ex, ey, i, j);
          x[g] = M.x0 + M.hx * ex + 0.5 * ((*sx)[i] + 1.0) * M.hx;
          y[g] = M.y0 + M.hy * ey + 0.5 * ((*sy)[j] + 1.0) * M.hy;
        }
  return 0;
}

// Connectivity of the periodic mesh.  nbr[K][4]: the neighbour across the left, right, bottom
// and top face.  dof (optional), concatenated:
//   face map [K][4][p+1]: for face f (left, right, bottom, top) and face node k (k indexes y on
//     x-normal faces, x on y-normal faces), the index e' (p+1)^2 + q' of the neighbour node at the
//     same point;
//   local-to-global maps [K][n_s] of the six magnetic node sets in the order B_x (GLL_{m+1} x
//     Gauss_m), B_y (Gauss_m x GLL_{m+1}), B_z (GLL_m^2), W (GLL_{m+1}^2), N_x (Gauss_m x
//     GLL_{m+1}), N_y (GLL_{m+1} x Gauss_m), local order [j][i], i fastest.
int or_get_maps(const int* im, const double* dm, int32_t* nbr, int32_t* dof) {
  Mesh M = make_mesh(im, dm);
  for (long e = 0; e < M.K; ++e) {
    const long ex = e % M.nx, ey = e / M.nx;
    nbr[4 * e + 0] = (int32_t)elem(M, ex - 1, ey);
    nbr[4 * e + 1] = (int32_t)elem(M, ex + 1, ey);
    nbr[4 * e + 2] = (int32_t)elem(M, ex, ey - 1);
    nbr[4 * e + 3] = (int32_t)elem(M, ex, ey + 1);
  }
  if (!dof) return 0;
  int32_t* o = dof;
  for (long e = 0; e < M.K; ++e) {
    const long ex = e % M.nx, ey = e / M.nx;
    for (int f = 0; f < 4; ++f)
      for (int k = 0; k < M.np; ++k) {
        long en;
        int i, j;  // the neighbour's node at the same point
        if (f == 0) { en = elem(M, ex - 1, ey); i = M.p; j = k; }
        else if (f == 1) { en = elem(M, ex + 1, ey); i = 0; j = k; }
        else if (f == 2) { en = elem(M, ex, ey - 1); i = k; j = M.p; }
        else { en = elem(M, ex, ey + 1); i = k; j = 0; }
        *o++ = (int32_t)nid(M, 0, en, i, j);
      }
  }
  const int A = M.m + 2, B = M.m + 1;
  const int ni[6] = {A, B, B, A, B, A}, nj[6] = {B, A, B, A, A, B};
  for (int s = 0; s < 6; ++s)
    for (long e = 0; e < M.K; ++e) {
      const long ex = e % M.nx, ey = e / M.nx;
      for (int j = 0; j < nj[s]; ++j)
        for (int i = 0; i < ni[s]; ++i) *o++ = (int32_t)gid(M, ex, ey, i, j);
    }
  return 0;
}

int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
