// Vector-Jacobian products of L_E and L_M for gfx950 (hand-derived reverse mode, stage
// recomputation, no stored Jacobians).  Hydro: the reverse of eq. euler-nodal-index with the
// pairwise Chandrashekar flux (eq. euler-chandrashekar-flux) and LLF interfaces (eq. euler-lf-flux)
// whose max/abs branches are taken at the forward state (ties: the minus side).  Magnetic: the
// transposes of the curl update, the Lorentz load, Ohmic heating and the J/E reconstructions
// (eq. magnetic-dae) with rho and eta frozen; shared degrees of freedom are summed by fixed-order
// gathers.
#include <cfloat>

#include "common.h"

namespace {

template <int P>
struct HC {
  static constexpr int NP = P + 1, NN = NP * NP, EB = 256 / NN, NT = EB * NN, ND = NP / 2;
};

struct Pr {
  double r, ux, uy, uz, b, lr, lb;
};

__device__ __forceinline__ Pr prim_of(const double U[5], double g) {
  Pr q;
  q.r = U[0];
  const double ir = 1.0 / U[0];
  q.ux = U[1] * ir; q.uy = U[2] * ir; q.uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * q.ux + U[2] * q.uy + U[3] * q.uz));
  q.b = 0.5 * q.r / p;
  q.lr = log(q.r); q.lb = log(q.b);
  return q;
}

// value and partial derivatives of the logarithmic mean (same branch rule as the forward)
__device__ __forceinline__ void lmean_d(double aL, double aR, double lL, double lR, double& v, double& gL, double& gR) {
  const double d = aR - aL, s = aR + aL;
  if (d * d < 1e-4 * (s * s)) {
    const double u = (d * d) / (s * s), f = d / s;
    const double h = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
    const double hp = 1.0 / 3.0 + u * (0.4 + u * (3.0 / 7.0));
    const double gg = 1.0 / h, gp = -hp * gg * gg;
    v = 0.5 * s * gg;
    gL = 0.5 * gg - 2.0 * f * aR * gp / s;
    gR = 0.5 * gg + 2.0 * f * aL * gp / s;
  } else {
    const double Lm = lR - lL;
    v = d / Lm;
    gL = (v / aL - 1.0) / Lm;
    gR = (1.0 - v / aR) / Lm;
  }
}

// reverse of the Chandrashekar flux: accumulates adjoints w.r.t. (rho, ux, uy, uz, beta) of both sides
template <int D>
__device__ __forceinline__ void ecflux_rev(const Pr& L, const Pr& R, double g, const double v[5], double bL[5],
                                           double bR[5]) {
  double rl, drL, drR, bl, dbL, dbR;
  lmean_d(L.r, R.r, L.lr, R.lr, rl, drL, drR);
  lmean_d(L.b, R.b, L.lb, R.lb, bl, dbL, dbR);
  const double sb = L.b + R.b;
  const double ph = 0.5 * (L.r + R.r) / sb;
  const double uxa = 0.5 * (L.ux + R.ux), uya = 0.5 * (L.uy + R.uy), uza = 0.5 * (L.uz + R.uz);
  const double u2a = 0.5 * ((L.ux * L.ux + L.uy * L.uy + L.uz * L.uz) + (R.ux * R.ux + R.uy * R.uy + R.uz * R.uz));
  const double ud = D == 0 ? uxa : uya;
  const double f0 = rl * ud;
  const double ig = 1.0 / (2.0 * (g - 1.0) * bl);
  const double H = ig - 0.5 * u2a + (uxa * uxa + uya * uya + uza * uza);
  const double f0b = v[0] + v[1] * uxa + v[2] * uya + v[3] * uza + v[4] * H;
  const double phb = (D == 0 ? v[1] : v[2]) + v[4] * ud;
  const double Hb = v[4] * f0;
  double uxab = v[1] * f0 + 2.0 * Hb * uxa;
  double uyab = v[2] * f0 + 2.0 * Hb * uya;
  const double uzab = v[3] * f0 + 2.0 * Hb * uza;
  const double udb = v[4] * ph + f0b * rl;
  if (D == 0) uxab += udb; else uyab += udb;
  const double rlb = f0b * ud;
  const double blb = -Hb * ig / bl;
  const double u2ab = -0.5 * Hb;
  const double phr = 0.5 / sb, phbeta = -ph / sb;
  bL[0] += phb * phr + rlb * drL;
  bR[0] += phb * phr + rlb * drR;
  bL[4] += phb * phbeta + blb * dbL;
  bR[4] += phb * phbeta + blb * dbR;
  bL[1] += 0.5 * uxab + u2ab * L.ux; bR[1] += 0.5 * uxab + u2ab * R.ux;
  bL[2] += 0.5 * uyab + u2ab * L.uy; bR[2] += 0.5 * uyab + u2ab * R.uy;
  bL[3] += 0.5 * uzab + u2ab * L.uz; bR[3] += 0.5 * uzab + u2ab * R.uz;
}

// adjoint of (rho, u, beta)(U) applied to prim adjoints pb, added to Ub
__device__ __forceinline__ void prim_rev(const double U[5], const double pb[5], double g, double Ub[5]) {
  const double r = U[0], ir = 1.0 / r;
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * ux + U[2] * uy + U[3] * uz));
  const double beta = 0.5 * r / p;
  const double rb = pb[0] + pb[4] * 0.5 / p;
  const double pbar = -pb[4] * beta / p;
  Ub[0] += rb + pbar * (g - 1.0) * 0.5 * (ux * ux + uy * uy + uz * uz) - (pb[1] * ux + pb[2] * uy + pb[3] * uz) * ir;
  Ub[1] += -pbar * (g - 1.0) * ux + pb[1] * ir;
  Ub[2] += -pbar * (g - 1.0) * uy + pb[2] * ir;
  Ub[3] += -pbar * (g - 1.0) * uz + pb[3] * ir;
  Ub[4] += pbar * (g - 1.0);
}

// pressure-adjoint chain p(rho, m, E)
__device__ __forceinline__ void p_rev(const double U[5], double pb, double g, double Ub[5]) {
  const double ir = 1.0 / U[0];
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  Ub[0] += pb * (g - 1.0) * 0.5 * (ux * ux + uy * uy + uz * uz);
  Ub[1] -= pb * (g - 1.0) * ux; Ub[2] -= pb * (g - 1.0) * uy; Ub[3] -= pb * (g - 1.0) * uz;
  Ub[4] += pb * (g - 1.0);
}

template <int D>
__device__ __forceinline__ void physflux_rev(const double U[5], double g, const double mu[5], double Ub[5]) {
  const double r = U[0], ir = 1.0 / r;
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * ux + U[2] * uy + U[3] * uz));
  const double ud = D == 0 ? ux : uy;
  Ub[1 + D] += mu[0];
  Ub[1] += mu[1] * ud; Ub[2] += mu[2] * ud; Ub[3] += mu[3] * ud; Ub[4] += mu[4] * ud;
  const double udb = mu[1] * U[1] + mu[2] * U[2] + mu[3] * U[3] + mu[4] * (U[4] + p);
  const double pb = (D == 0 ? mu[1] : mu[2]) + mu[4] * ud;
  Ub[1 + D] += udb * ir;
  Ub[0] -= udb * ud * ir;
  p_rev(U, pb, g, Ub);
}

template <int D>
__device__ __forceinline__ double speed(const double U[5], double g) {
  const double ir = 1.0 / U[0];
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * ux + U[2] * uy + U[3] * uz));
  return fabs(D == 0 ? ux : uy) + sqrt(g * p * ir);
}

template <int D>
__device__ __forceinline__ void speed_rev(const double U[5], double g, double sb, double Ub[5]) {
  const double r = U[0], ir = 1.0 / r;
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * ux + U[2] * uy + U[3] * uz));
  const double ud = D == 0 ? ux : uy;
  const double c = sqrt(g * p * ir);
  const double udb = sb * (ud < 0.0 ? -1.0 : 1.0);
  Ub[1 + D] += udb * ir;
  Ub[0] -= udb * ud * ir;
  const double pb = sb * g / (2.0 * c * r);
  Ub[0] += -sb * c / (2.0 * r);
  p_rev(U, pb, g, Ub);
}

// reverse of the interface flux F*(UL, UR) for the element's own side
template <int D>
__device__ __forceinline__ void iflux_rev(const double UL[5], const double UR[5], double g, int iface,
                                          const double mu[5], bool own_left, double Ub[5]) {
  if (iface == 1) {
    Pr a = prim_of(UL, g), b = prim_of(UR, g);
    double pa[5] = {0, 0, 0, 0, 0}, pbv[5] = {0, 0, 0, 0, 0};
    ecflux_rev<D>(a, b, g, mu, pa, pbv);
    if (own_left) prim_rev(UL, pa, g, Ub); else prim_rev(UR, pbv, g, Ub);
    return;
  }
  const double sL = speed<D>(UL, g), sR = speed<D>(UR, g);
  const bool left_wins = sL >= sR;
  const double lam = left_wins ? sL : sR;
  double dot = 0.0;
#pragma unroll
  for (int c = 0; c < 5; ++c) dot += mu[c] * (UR[c] - UL[c]);
  double h[5] = {0.5 * mu[0], 0.5 * mu[1], 0.5 * mu[2], 0.5 * mu[3], 0.5 * mu[4]};
  if (own_left) {
    physflux_rev<D>(UL, g, h, Ub);
#pragma unroll
    for (int c = 0; c < 5; ++c) Ub[c] += 0.5 * lam * mu[c];
    if (left_wins) speed_rev<D>(UL, g, -0.5 * dot, Ub);
  } else {
    physflux_rev<D>(UR, g, h, Ub);
#pragma unroll
    for (int c = 0; c < 5; ++c) Ub[c] -= 0.5 * lam * mu[c];
    if (!left_wins) speed_rev<D>(UR, g, -0.5 * dot, Ub);
  }
}

__device__ __forceinline__ long wrap(long a, long n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

template <int P, int D>
__device__ __forceinline__ void vjp_dir(const Pr& me, const double U[5], const double lam[5], double pbo[5],
                                        double Ub[5], bool act, int el, int i, int j, long e,
                                        const double* __restrict__ Us, const double* __restrict__ cot, long KN,
                                        double (*sp)[HC<P>::EB * HC<P>::NN], double (*sl)[HC<P>::EB * HC<P>::NN],
                                        double* sb, const HydroTab* __restrict__ T, const MeshP& mp, int iface) {
  using C = HC<P>;
  constexpr int NP = C::NP, NN = C::NN, ND = C::ND;
  const int pos = D == 0 ? i : j, line = D == 0 ? j : i;
  const double sc = D == 0 ? 2.0 / mp.hx : 2.0 / mp.hy;
  const double g = mp.gamma;
  double* sbl = sb + ((long)(el * NP + line) * NP) * ND * 5;
  if (act) {
#pragma unroll
    for (int d = 1; d <= ND; ++d) {
      if (2 * d == NP && pos >= NP / 2) continue;
      int r = pos + d;
      if (r >= NP) r -= NP;
      const int nr = el * NN + (D == 0 ? line * NP + r : r * NP + line);
      Pr o;
      o.r = sp[0][nr]; o.ux = sp[1][nr]; o.uy = sp[2][nr]; o.uz = sp[3][nr];
      o.b = sp[4][nr]; o.lr = sp[5][nr]; o.lb = sp[6][nr];
      const double ci = -sc * T->Shat[pos][r], cr = -sc * T->Shat[r][pos];
      double v[5], bo[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int c = 0; c < 5; ++c) v[c] = ci * lam[c] + cr * sl[c][nr];
      ecflux_rev<D>(me, o, g, v, pbo, bo);
#pragma unroll
      for (int c = 0; c < 5; ++c) sbl[(pos * ND + (d - 1)) * 5 + c] = bo[c];
    }
    if (pos == 0 || pos == P) {
      long ex, ey;
      elem_xy(mp, e, ex, ey);
      long en;
      if (D == 0) en = ey * mp.nx + wrap(ex + (pos == 0 ? -1 : 1), mp.nx);
      else en = wrap(ey + (pos == 0 ? -1 : 1), mp.ny) * mp.nx + ex;
      const int qn = D == 0 ? line * NP + (pos == 0 ? P : 0) : (pos == 0 ? P : 0) * NP + line;
      double UN[5], mu[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) UN[c] = Us[c * KN + en * NN + qn];
      if (pos == 0) {  // own is the plus side of the face
#pragma unroll
        for (int c = 0; c < 5; ++c) mu[c] = (sc / T->w[0]) * lam[c] - (sc / T->w[P]) * cot[c * KN + en * NN + qn];
        iflux_rev<D>(UN, U, g, iface, mu, false, Ub);
      } else {  // own is the minus side
#pragma unroll
        for (int c = 0; c < 5; ++c) mu[c] = -(sc / T->w[P]) * lam[c] + (sc / T->w[0]) * cot[c * KN + en * NN + qn];
        iflux_rev<D>(U, UN, g, iface, mu, true, Ub);
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int d = 1; d <= ND; ++d) {
      int o = pos - d;
      if (o < 0) o += NP;
      if (2 * d == NP && o >= NP / 2) continue;
#pragma unroll
      for (int c = 0; c < 5; ++c) pbo[c] += sbl[(o * ND + (d - 1)) * 5 + c];
    }
  }
  __syncthreads();
}

template <int P>
__global__ __launch_bounds__(256) void k_hydro_vjp(const double* __restrict__ Us, const double* __restrict__ cot,
                                                   double* __restrict__ Ubar, const HydroTab* __restrict__ T, MeshP mp,
                                                   int iface) {
  using C = HC<P>;
  constexpr int NP = C::NP, NN = C::NN, EB = C::EB, ND = C::ND;
  __shared__ double sp[7][EB * NN];
  __shared__ double sl[5][EB * NN];
  __shared__ double sb[EB * NP * NP * (ND > 0 ? ND : 1) * 5];
  const int tid = threadIdx.x;
  const int el = tid / NN, q = tid - el * NN;
  const int i = q % NP, j = q / NP;
  const long e = (long)blockIdx.x * EB + el;
  const bool act = tid < C::NT && e < mp.K;
  const long KN = mp.K * NN;
  double U[5], lam[5], pbo[5] = {0, 0, 0, 0, 0}, Ub[5] = {0, 0, 0, 0, 0};
  Pr me{};
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) { U[c] = Us[c * KN + e * NN + q]; lam[c] = cot[c * KN + e * NN + q]; sl[c][tid] = lam[c]; }
    me = prim_of(U, mp.gamma);
    sp[0][tid] = me.r; sp[1][tid] = me.ux; sp[2][tid] = me.uy; sp[3][tid] = me.uz;
    sp[4][tid] = me.b; sp[5][tid] = me.lr; sp[6][tid] = me.lb;
  }
  __syncthreads();
  vjp_dir<P, 0>(me, U, lam, pbo, Ub, act, el, i, j, e, Us, cot, KN, sp, sl, sb, T, mp, iface);
  vjp_dir<P, 1>(me, U, lam, pbo, Ub, act, el, i, j, e, Us, cot, KN, sp, sl, sb, T, mp, iface);
  if (act) {
    prim_rev(U, pbo, mp.gamma, Ub);
#pragma unroll
    for (int c = 0; c < 5; ++c) Ubar[c * KN + e * NN + q] = Ub[c];
  }
}

// ---------------------------------------------------------------------------------------------
// magnetic VJP
// ---------------------------------------------------------------------------------------------
template <int P, int M>
struct MV {
  static constexpr int NP = P + 1, NN = NP * NP, A = M + 2, B = M + 1, AA = A * A, AB = A * B, BB = B * B;
  static constexpr int NT = NN > AA ? NN : AA;
  static constexpr int EB = 256 / NT;
  static constexpr int LOC = 2 * AB + AA;  // one set of local arrays in (Nx, Ny, W) layouts
};

__device__ __forceinline__ long gix(const MeshP& mp, int B, long ex, long ey, int i, int j) {
  const long NX = (long)mp.nx * B, NY = (long)mp.ny * B;
  long gx = ex * B + i, gy = ey * B + j;
  if (gx >= NX) gx -= NX;
  if (gy >= NY) gy -= NY;
  return gy * NX + gx;
}

// Reverse of the update (curl, Lorentz, Ohm).  Writes per-element locals:
//   EL: E-bar in (Nx, Ny, W) layouts; JL: J-bar (Lorentz + Ohm) in (Nx, Ny, W);
//   BL: B-bar of the element's B locals: [bx: Ny layout (AB) | by: Nx layout (AB) | bz (BB)] (accumulated).
template <int P, int M>
__global__ __launch_bounds__(256) void k_vjp_update(const double* __restrict__ rho, const double* __restrict__ Bx,
                                                    const double* __restrict__ By, const double* __restrict__ Bz,
                                                    const double* __restrict__ JE, const double* __restrict__ eta,
                                                    const double* __restrict__ de_c, const double* __restrict__ du_c,
                                                    const double* __restrict__ dBx_c, const double* __restrict__ dBy_c,
                                                    const double* __restrict__ dBz_c, double* __restrict__ EL,
                                                    double* __restrict__ JL, double* __restrict__ BL,
                                                    const MagTab* __restrict__ T, MeshP mp, long G) {
  using C = MV<P, M>;
  constexpr int NP = C::NP, NN = C::NN, A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB,
                NT = C::NT, LOC = C::LOC;
  __shared__ double sbx[EB][AB], sby[EB][AB], sbz[EB][BB], sjx[EB][AB], sjy[EB][AB], sjz[EB][AA];
  __shared__ double scx[EB][BB], scy[EB][BB], scz[EB][BB];  // cotangents at owned B nodes
  __shared__ double sup[EB][3][NN];                         // du_cot / (rho M)
  __shared__ double sjq[EB][3][NN];                         // J-bar at GLL_p nodes (Ohm)
  __shared__ double sfb[EB][3][AA + 2 * AB];                // B-bar at aux nodes: W (AA), Nx (AB), Ny (AB)
  // the interpolation and derivative tables, staged in LDS (lane-dependent indexes into the
  // device table would each be a vector memory load)
  __shared__ double tDWG[MHD_MAXN][MHD_MAXN], tDWV[MHD_MAXN][MHD_MAXN], tIGP[MHD_MAXN][MHD_MAXN], tIGV[MHD_MAXN][MHD_MAXN], tIGW[MHD_MAXN][MHD_MAXN], tIVG[MHD_MAXN][MHD_MAXN], tIVW[MHD_MAXN][MHD_MAXN], tIWP[MHD_MAXN][MHD_MAXN], tIPW[MHD_MAXN][MHD_MAXN], tIPG[MHD_MAXN][MHD_MAXN];
  __shared__ double tww[MHD_MAXN], twg[MHD_MAXN], twp[MHD_MAXN];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  for (int k = threadIdx.x; k < MHD_MAXN * MHD_MAXN; k += 256) {
    const int r = k / MHD_MAXN, c = k % MHD_MAXN;
    tDWG[r][c] = T->D_W_G[r][c];
    tDWV[r][c] = T->D_W_V[r][c];
    tIGP[r][c] = T->I_G_P[r][c];
    tIGV[r][c] = T->I_G_V[r][c];
    tIGW[r][c] = T->I_G_W[r][c];
    tIVG[r][c] = T->I_V_G[r][c];
    tIVW[r][c] = T->I_V_W[r][c];
    tIWP[r][c] = T->I_W_P[r][c];
    tIPW[r][c] = T->I_P_W[r][c];
    tIPG[r][c] = T->I_P_G[r][c];
  }
  if (threadIdx.x < MHD_MAXN) { tww[threadIdx.x] = T->ww[threadIdx.x]; twg[threadIdx.x] = T->wg[threadIdx.x]; twp[threadIdx.x] = T->wp[threadIdx.x]; }
  __syncthreads();  // the load phase below already reads the tables
  const long e = (long)blockIdx.x * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  const double et = (act && eta) ? eta[e] : 0.0;
  const double* Jx = JE; const double* Jy = JE + G; const double* Jz = JE + 2 * G;
  if (act) {
    for (int k = t; k < AB; k += NT) {
      sbx[el][k] = Bx[gix(mp, B, ex, ey, k % A, k / A)];
      sby[el][k] = By[gix(mp, B, ex, ey, k % B, k / B)];
      sjx[el][k] = Jx[gix(mp, B, ex, ey, k % B, k / B)];
      sjy[el][k] = Jy[gix(mp, B, ex, ey, k % A, k / A)];
    }
    for (int k = t; k < AA; k += NT) sjz[el][k] = Jz[gix(mp, B, ex, ey, k % A, k / A)];
    for (int k = t; k < BB; k += NT) {
      const long g = gix(mp, B, ex, ey, k % B, k / B);
      sbz[el][k] = Bz[g];
      scx[el][k] = dBx_c[g]; scy[el][k] = dBy_c[g]; scz[el][k] = dBz_c[g];
    }
    if (t < NN) {
      const int qi = t % NP, qj = t / NP;
      const long n = e * NN + t;
      const double w = 1.0 / (rho[n] * mp.J * twp[qi] * twp[qj]);
      for (int d = 0; d < 3; ++d) sup[el][d][t] = du_c[d * KN + n] * w;
      // Ohm: de = eta |J(x_q)|^2 / rho  ->  J-bar(x_q) = de_c * 2 eta J / rho
      double jx = 0.0, jy = 0.0, jz = 0.0;
      if (et != 0.0) {
        for (int jj = 0; jj < A; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < B; ++ii) s += tIGP[qi][ii] * Jx[gix(mp, B, ex, ey, ii, jj)];
          jx += tIWP[qj][jj] * s;
        }
        for (int jj = 0; jj < B; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < A; ++ii) s += tIWP[qi][ii] * Jy[gix(mp, B, ex, ey, ii, jj)];
          jy += tIGP[qj][jj] * s;
        }
        for (int jj = 0; jj < A; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < A; ++ii) s += tIWP[qi][ii] * Jz[gix(mp, B, ex, ey, ii, jj)];
          jz += tIWP[qj][jj] * s;
        }
      }
      const double f = et != 0.0 ? de_c[n] * 2.0 * et / rho[n] : 0.0;
      sjq[el][0][t] = f * jx; sjq[el][1][t] = f * jy; sjq[el][2][t] = f * jz;
    }
  }
  __syncthreads();
  double* ELe = EL + e * LOC;
  double* JLe = JL + e * LOC;
  double* BLe = BL + e * (2 * AB + BB);
  if (act) {
    // E-bar from the curl (owned B nodes only; E nodes of the element's last GLL row/column belong to
    // neighbours' B nodes and receive nothing from this element)
    if (t < AA) {  // E_z local (i, k) = column i, row k
      const int i = t % A, k = t / A;
      double s = 0.0;
      if (i < B)
        for (int j = 0; j < B; ++j) s += -(2.0 / mp.hy) * tDWG[j][k] * scx[el][j * B + i];
      if (k < B)
        for (int ii = 0; ii < B; ++ii) s += (2.0 / mp.hx) * tDWG[ii][i] * scy[el][k * B + ii];
      ELe[2 * AB + t] = s;
    }
    if (t < AB) {
      {  // E_y local: Ny layout (i < A GLL x, l < B Gauss y); dBz = -(2/hx) sum I_G_V[j][l] D_W_V[i'][i] E_y
        const int i = t % A, l = t / A;
        double s = 0.0;
        for (int jj = 0; jj < B; ++jj)
          for (int ii = 0; ii < B; ++ii) s += tIGV[jj][l] * tDWV[ii][i] * scz[el][jj * B + ii];
        ELe[AB + t] = -(2.0 / mp.hx) * s;
      }
      {  // E_x local: Nx layout (k < B Gauss x, l < A GLL y); dBz += (2/hy) sum D_W_V[j][l] I_G_V[i][k] E_x
        const int k = t % B, l = t / B;
        double s = 0.0;
        for (int jj = 0; jj < B; ++jj)
          for (int ii = 0; ii < B; ++ii) s += tDWV[jj][l] * tIGV[ii][k] * scz[el][jj * B + ii];
        ELe[t] = (2.0 / mp.hy) * s;
      }
    }
    // Lorentz reverse at aux nodes: f-bar_a = w_a sum_q I_{a,q} u'_q
    auto fbar = [&](int d, const double (*Ix)[MHD_MAXN], int ai, const double (*Iy)[MHD_MAXN], int aj) {
      double v = 0.0;
      for (int qj = 0; qj < NP; ++qj) {
        double s = 0.0;
        for (int qi = 0; qi < NP; ++qi) s += Ix[ai][qi] * sup[el][d][qj * NP + qi];
        v += Iy[aj][qj] * s;
      }
      return v;
    };
    // Ohm reverse J-bar at aux node a of one layout: sum_q phi_a(x_q) Jbar(x_q)
    auto ohm = [&](int c, const double (*Px)[MHD_MAXN], int ai, const double (*Py)[MHD_MAXN], int aj) {
      double v = 0.0;
      for (int qj = 0; qj < NP; ++qj)
        for (int qi = 0; qi < NP; ++qi) v += sjq[el][c][qj * NP + qi] * (Px[qi][ai] * Py[qj][aj]);
      return v;
    };
    if (t < AA) {  // W node: f = (-B_y J_z, B_x J_z, 0)
      const int i = t % A, j = t / A;
      const double w = mp.J * tww[i] * tww[j];
      const double fx = w * fbar(0, tIPW, i, tIPW, j), fy = w * fbar(1, tIPW, i, tIPW, j);
      double bxv = 0.0, byv = 0.0;
      for (int k = 0; k < B; ++k) { bxv += tIGW[j][k] * sbx[el][k * A + i]; byv += tIGW[i][k] * sby[el][j * B + k]; }
      const double jz = sjz[el][t];
      JLe[2 * AB + t] = -fx * byv + fy * bxv + (et != 0.0 ? ohm(2, tIWP, i, tIWP, j) : 0.0);
      sfb[el][0][t] = fy * jz;   // B_x bar at W node
      sfb[el][1][t] = -fx * jz;  // B_y bar
      sfb[el][2][t] = 0.0;
    }
    if (t < AB) {
      {  // N_x node (i < B, j < A): f = (0, -B_z J_x, B_y J_x)
        const int i = t % B, j = t / B;
        const double w = mp.J * twg[i] * tww[j];
        const double fy = w * fbar(1, tIPG, i, tIPW, j), fz = w * fbar(2, tIPG, i, tIPW, j);
        double bzv = 0.0;
        for (int jj = 0; jj < B; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < B; ++ii) s += tIVG[i][ii] * sbz[el][jj * B + ii];
          bzv += tIVW[j][jj] * s;
        }
        const double jx = sjx[el][t];
        JLe[t] = -fy * bzv + fz * sby[el][t] + (et != 0.0 ? ohm(0, tIGP, i, tIWP, j) : 0.0);
        sfb[el][0][AA + t] = 0.0;
        sfb[el][1][AA + t] = fz * jx;   // B_y bar (B_y lives on these nodes)
        sfb[el][2][AA + t] = -fy * jx;  // B_z bar at the node
      }
      {  // N_y node (i < A, j < B): f = (B_z J_y, 0, -B_x J_y)
        const int i = t % A, j = t / A;
        const double w = mp.J * tww[i] * twg[j];
        const double fx = w * fbar(0, tIPW, i, tIPG, j), fz = w * fbar(2, tIPW, i, tIPG, j);
        double bzv = 0.0;
        for (int jj = 0; jj < B; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < B; ++ii) s += tIVW[i][ii] * sbz[el][jj * B + ii];
          bzv += tIVG[j][jj] * s;
        }
        const double jy = sjy[el][t];
        JLe[AB + t] = fx * bzv - fz * sbx[el][t] + (et != 0.0 ? ohm(1, tIWP, i, tIGP, j) : 0.0);
        sfb[el][0][AA + AB + t] = -fz * jy;  // B_x bar (B_x lives on these nodes)
        sfb[el][1][AA + AB + t] = 0.0;
        sfb[el][2][AA + AB + t] = fx * jy;   // B_z bar
      }
    }
  }
  __syncthreads();
  if (!act) return;
  // transpose-interpolate aux-node B-bar to the element's B locals
  if (t < AB) {
    {  // B_x local (i < A, k < B): from W nodes (i, j) via I_G_W[j][k] and from N_y node t directly
      const int i = t % A, k = t / A;
      double s = sfb[el][0][AA + AB + t];
      for (int j = 0; j < A; ++j) s += tIGW[j][k] * sfb[el][0][j * A + i];
      BLe[t] = s;
    }
    {  // B_y local (k < B, j < A): from W nodes (i, j) via I_G_W[i][k] and from N_x node t directly
      const int k = t % B, j = t / B;
      double s = sfb[el][1][AA + t];
      for (int i = 0; i < A; ++i) s += tIGW[i][k] * sfb[el][1][j * A + i];
      BLe[AB + t] = s;
    }
  }
  if (t < BB) {  // B_z local (ii, jj): from N_x (I_V_G x, I_V_W y) and N_y (I_V_W x, I_V_G y)
    const int ii = t % B, jj = t / B;
    double s = 0.0;
    for (int j = 0; j < A; ++j)
      for (int i = 0; i < B; ++i) s += tIVG[i][ii] * tIVW[j][jj] * sfb[el][2][AA + j * B + i];
    for (int j = 0; j < B; ++j)
      for (int i = 0; i < A; ++i) s += tIVW[i][ii] * tIVG[j][jj] * sfb[el][2][AA + AB + j * A + i];
    BLe[2 * AB + t] = s;
  }
}

// Reverse of the E reconstruction: given E-bar (grids), produce u-bar (direct), and add
// B-bar locals and J-bar locals (eta term).
template <int P, int M>
__global__ __launch_bounds__(256) void k_vjp_E(const double* __restrict__ u, const double* __restrict__ Bx,
                                               const double* __restrict__ By, const double* __restrict__ Bz,
                                               const double* __restrict__ Ebar, const double* __restrict__ eta,
                                               double* __restrict__ ubar, double* __restrict__ JL,
                                               double* __restrict__ BL, const MagTab* __restrict__ T, MeshP mp,
                                               long G) {
  using C = MV<P, M>;
  constexpr int NP = C::NP, NN = C::NN, A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB,
                NT = C::NT, LOC = C::LOC;
  __shared__ double su[EB][3][NN], sbx[EB][AB], sby[EB][AB], sbz[EB][BB];
  __shared__ double sl[EB][AA + 2 * AB];          // load-bar = E-bar / m at the element's aux nodes (W, Nx, Ny)
  __shared__ double sub[EB][3][AA + 2 * AB];      // u-bar at aux nodes
  __shared__ double sbb[EB][3][AA + 2 * AB];      // B-bar at aux nodes
  __shared__ double tWP[NP][A], tGP[NP][B];         // W and Gauss bases at the GLL_p nodes (eta term)
  // the interpolation tables, staged in LDS (lane-dependent indexes into the device table would
  // each be a vector memory load)
  __shared__ double tIGW[MHD_MAXN][MHD_MAXN], tIPG[MHD_MAXN][MHD_MAXN], tIPW[MHD_MAXN][MHD_MAXN], tIVG[MHD_MAXN][MHD_MAXN], tIVW[MHD_MAXN][MHD_MAXN];
  __shared__ double tww[MHD_MAXN], twg[MHD_MAXN], twp[MHD_MAXN];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  for (int k = tid; k < NP * A; k += 256) tWP[k / A][k % A] = T->I_W_P[k / A][k % A];
  for (int k = tid; k < NP * B; k += 256) tGP[k / B][k % B] = T->I_G_P[k / B][k % B];
  for (int k = tid; k < MHD_MAXN * MHD_MAXN; k += 256) {
    const int r = k / MHD_MAXN, c = k % MHD_MAXN;
    tIGW[r][c] = T->I_G_W[r][c];
    tIPG[r][c] = T->I_P_G[r][c];
    tIPW[r][c] = T->I_P_W[r][c];
    tIVG[r][c] = T->I_V_G[r][c];
    tIVW[r][c] = T->I_V_W[r][c];
  }
  if (tid < MHD_MAXN) { tww[tid] = T->ww[tid]; twg[tid] = T->wg[tid]; twp[tid] = T->wp[tid]; }
  __syncthreads();  // the load phase below already reads the tables
  const long e = (long)blockIdx.x * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  const double et = (act && eta) ? eta[e] : 0.0;
  const double* Exb = Ebar; const double* Eyb = Ebar + G; const double* Ezb = Ebar + 2 * G;
  if (act) {
    for (int k = t; k < NN; k += NT)
      for (int d = 0; d < 3; ++d) su[el][d][k] = u[d * KN + e * NN + k];
    for (int k = t; k < AB; k += NT) {
      sbx[el][k] = Bx[gix(mp, B, ex, ey, k % A, k / A)];
      sby[el][k] = By[gix(mp, B, ex, ey, k % B, k / B)];
    }
    for (int k = t; k < BB; k += NT) sbz[el][k] = Bz[gix(mp, B, ex, ey, k % B, k / B)];
    // load-bar = E-bar / (assembled lumped weight); weights are sums over the sharing elements
    for (int k = t; k < AA; k += NT) {
      const int i = k % A, j = k / A;
      const double wx = (i == 0 || i == A - 1) ? tww[0] + tww[A - 1] : tww[i];
      const double wy = (j == 0 || j == A - 1) ? tww[0] + tww[A - 1] : tww[j];
      sl[el][k] = Ezb[gix(mp, B, ex, ey, i, j)] / (mp.J * wx * wy);
    }
    for (int k = t; k < AB; k += NT) {
      {
        const int i = k % B, j = k / B;  // Nx
        const double wy = (j == 0 || j == A - 1) ? tww[0] + tww[A - 1] : tww[j];
        sl[el][AA + k] = Exb[gix(mp, B, ex, ey, i, j)] / (mp.J * twg[i] * wy);
      }
      {
        const int i = k % A, j = k / A;  // Ny
        const double wx = (i == 0 || i == A - 1) ? tww[0] + tww[A - 1] : tww[i];
        sl[el][AA + AB + k] = Eyb[gix(mp, B, ex, ey, i, j)] / (mp.J * wx * twg[j]);
      }
    }
  }
  __syncthreads();
  auto u_at = [&](int d, const double (*Ix)[MHD_MAXN], int ai, const double (*Iy)[MHD_MAXN], int aj) {
    double v = 0.0;
    for (int qj = 0; qj < NP; ++qj) {
      double s = 0.0;
      for (int qi = 0; qi < NP; ++qi) s += Ix[ai][qi] * su[el][d][qj * NP + qi];
      v += Iy[aj][qj] * s;
    }
    return v;
  };
  if (act) {
    if (t < AA) {  // W node: X_z = -(u_x B_y - u_y B_x)
      const int i = t % A, j = t / A;
      const double ux = u_at(0, tIPW, i, tIPW, j), uy = u_at(1, tIPW, i, tIPW, j);
      double bxv = 0.0, byv = 0.0;
      for (int k = 0; k < B; ++k) { bxv += tIGW[j][k] * sbx[el][k * A + i]; byv += tIGW[i][k] * sby[el][j * B + k]; }
      const double s = mp.J * tww[i] * tww[j] * sl[el][t];
      sub[el][0][t] = -s * byv; sub[el][1][t] = s * bxv; sub[el][2][t] = 0.0;
      sbb[el][0][t] = s * uy; sbb[el][1][t] = -s * ux; sbb[el][2][t] = 0.0;
    }
    if (t < AB) {
      {  // N_x node: X_x = -(u_y B_z - u_z B_y)
        const int i = t % B, j = t / B;
        const double uy = u_at(1, tIPG, i, tIPW, j), uz = u_at(2, tIPG, i, tIPW, j);
        const double byv = sby[el][t];
        double bzv = 0.0;
        for (int jj = 0; jj < B; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < B; ++ii) s += tIVG[i][ii] * sbz[el][jj * B + ii];
          bzv += tIVW[j][jj] * s;
        }
        const double s = mp.J * twg[i] * tww[j] * sl[el][AA + t];
        sub[el][0][AA + t] = 0.0; sub[el][1][AA + t] = -s * bzv; sub[el][2][AA + t] = s * byv;
        sbb[el][0][AA + t] = 0.0; sbb[el][1][AA + t] = s * uz; sbb[el][2][AA + t] = -s * uy;
      }
      {  // N_y node: X_y = -(u_z B_x - u_x B_z)
        const int i = t % A, j = t / A;
        const double ux = u_at(0, tIPW, i, tIPG, j), uz = u_at(2, tIPW, i, tIPG, j);
        const double bxv = sbx[el][t];
        double bzv = 0.0;
        for (int jj = 0; jj < B; ++jj) {
          double s = 0.0;
          for (int ii = 0; ii < B; ++ii) s += tIVW[i][ii] * sbz[el][jj * B + ii];
          bzv += tIVG[j][jj] * s;
        }
        const double s = mp.J * tww[i] * twg[j] * sl[el][AA + AB + t];
        sub[el][0][AA + AB + t] = s * bzv; sub[el][1][AA + AB + t] = 0.0; sub[el][2][AA + AB + t] = -s * bxv;
        sbb[el][0][AA + AB + t] = -s * uz; sbb[el][1][AA + AB + t] = 0.0; sbb[el][2][AA + AB + t] = s * ux;
      }
    }
  }
  // eta term: load_a += eta sum_q M_q J_c(x_q) phi_a(x_q), so J-bar_c(x_q) = eta M_q sum_a phi_a(x_q)
  // lbar_a; it is formed once per GLL_p node (into su, whose last reads precede this barrier) and
  // then moved to the J-bar locals by the transpose of the J interpolation to GLL_p
  const int any_eta = __syncthreads_or(act && et != 0.0);
  if (any_eta) {
    if (act && et != 0.0 && t < NN) {
      const int qi = t % NP, qj = t / NP;
      double vz = 0.0, vx = 0.0, vy = 0.0;
      for (int j = 0; j < A; ++j)
        for (int i = 0; i < A; ++i) vz += tWP[qi][i] * tWP[qj][j] * sl[el][j * A + i];
      for (int j = 0; j < A; ++j)
        for (int i = 0; i < B; ++i) vx += tGP[qi][i] * tWP[qj][j] * sl[el][AA + j * B + i];
      for (int j = 0; j < B; ++j)
        for (int i = 0; i < A; ++i) vy += tWP[qi][i] * tGP[qj][j] * sl[el][AA + AB + j * A + i];
      const double wq = et * mp.J * twp[qi] * twp[qj];
      su[el][0][t] = wq * vx; su[el][1][t] = wq * vy; su[el][2][t] = wq * vz;
    }
    __syncthreads();
  }
  if (!act) return;
  double* JLe = JL + e * LOC;
  double* BLe = BL + e * (2 * AB + BB);
  if (t < NN) {  // u-bar at GLL_p node q: transpose of the three interpolations
    const int qi = t % NP, qj = t / NP;
    for (int d = 0; d < 3; ++d) {
      double s = 0.0;
      for (int j = 0; j < A; ++j)
        for (int i = 0; i < A; ++i) s += tIPW[i][qi] * tIPW[j][qj] * sub[el][d][j * A + i];
      for (int j = 0; j < A; ++j)
        for (int i = 0; i < B; ++i) s += tIPG[i][qi] * tIPW[j][qj] * sub[el][d][AA + j * B + i];
      for (int j = 0; j < B; ++j)
        for (int i = 0; i < A; ++i) s += tIPW[i][qi] * tIPG[j][qj] * sub[el][d][AA + AB + j * A + i];
      ubar[d * KN + e * NN + t] = s;
    }
  }
  if (t < AB) {
    {  // B_x local (i < A, k < B)
      const int i = t % A, k = t / A;
      double s = sbb[el][0][AA + AB + t];
      for (int j = 0; j < A; ++j) s += tIGW[j][k] * sbb[el][0][j * A + i];
      BLe[t] += s;
    }
    {  // B_y local (k < B, j < A)
      const int k = t % B, j = t / B;
      double s = sbb[el][1][AA + t];
      for (int i = 0; i < A; ++i) s += tIGW[i][k] * sbb[el][1][j * A + i];
      BLe[AB + t] += s;
    }
  }
  if (t < BB) {
    const int ii = t % B, jj = t / B;
    double s = 0.0;
    for (int j = 0; j < A; ++j)
      for (int i = 0; i < B; ++i) s += tIVG[i][ii] * tIVW[j][jj] * sbb[el][2][AA + j * B + i];
    for (int j = 0; j < B; ++j)
      for (int i = 0; i < A; ++i) s += tIVW[i][ii] * tIVG[j][jj] * sbb[el][2][AA + AB + j * A + i];
    BLe[2 * AB + t] += s;
  }
  if (et != 0.0) {
    const double(*jq)[NN] = su[el];  // J-bar_x, J-bar_y, J-bar_z at the GLL_p nodes
    if (t < AA) {
      const int i = t % A, j = t / A;
      double s = 0.0;
      for (int qj = 0; qj < NP; ++qj)
        for (int qi = 0; qi < NP; ++qi) s += tWP[qi][i] * tWP[qj][j] * jq[2][qj * NP + qi];
      JLe[2 * AB + t] += s;
    }
    if (t < AB) {
      {
        const int i = t % B, j = t / B;
        double s = 0.0;
        for (int qj = 0; qj < NP; ++qj)
          for (int qi = 0; qi < NP; ++qi) s += tGP[qi][i] * tWP[qj][j] * jq[0][qj * NP + qi];
        JLe[t] += s;
      }
      {
        const int i = t % A, j = t / A;
        double s = 0.0;
        for (int qj = 0; qj < NP; ++qj)
          for (int qi = 0; qi < NP; ++qi) s += tWP[qi][i] * tGP[qj][j] * jq[1][qj * NP + qi];
        JLe[AB + t] += s;
      }
    }
  }
}

// Reverse of the J reconstruction: given J-bar (grids) add the B-bar locals of the weak curl.
template <int P, int M>
__global__ __launch_bounds__(256) void k_vjp_J(const double* __restrict__ Jbar, double* __restrict__ BL,
                                               const MagTab* __restrict__ T, MeshP mp, long G) {
  using C = MV<P, M>;
  constexpr int A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB, NT = C::NT;
  __shared__ double lz[EB][AA], lx[EB][AB], ly[EB][AB];
  __shared__ double qx_[EB][AA], qy_[EB][AA], zg[EB][BB];
  // the interpolation and derivative tables, staged in LDS (lane-dependent indexes into the device
  // table would each be a vector memory load)
  __shared__ double tDWG[MHD_MAXN][MHD_MAXN], tDWQ[MHD_MAXN][MHD_MAXN], tIGQ[MHD_MAXN][MHD_MAXN], tIVG[MHD_MAXN][MHD_MAXN], tIWQ[MHD_MAXN][MHD_MAXN];
  __shared__ double tww[MHD_MAXN], twg[MHD_MAXN], twq[MHD_MAXN];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  for (int k = tid; k < MHD_MAXN * MHD_MAXN; k += 256) {
    const int r = k / MHD_MAXN, c = k % MHD_MAXN;
    tDWG[r][c] = T->D_W_G[r][c];
    tDWQ[r][c] = T->D_W_Q[r][c];
    tIGQ[r][c] = T->I_G_Q[r][c];
    tIVG[r][c] = T->I_V_G[r][c];
    tIWQ[r][c] = T->I_W_Q[r][c];
  }
  if (tid < MHD_MAXN) { tww[tid] = T->ww[tid]; twg[tid] = T->wg[tid]; twq[tid] = T->wq[tid]; }
  __syncthreads();  // the load phase below already reads the tables
  const long e = (long)blockIdx.x * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const double* Jxb = Jbar; const double* Jyb = Jbar + G; const double* Jzb = Jbar + 2 * G;
  if (act) {
    for (int k = t; k < AA; k += NT) {
      const int i = k % A, j = k / A;
      const double wx = (i == 0 || i == A - 1) ? tww[0] + tww[A - 1] : tww[i];
      const double wy = (j == 0 || j == A - 1) ? tww[0] + tww[A - 1] : tww[j];
      lz[el][k] = Jzb[gix(mp, B, ex, ey, i, j)] / (mp.J * wx * wy);
    }
    for (int k = t; k < AB; k += NT) {
      {
        const int i = k % B, j = k / B;
        const double wy = (j == 0 || j == A - 1) ? tww[0] + tww[A - 1] : tww[j];
        lx[el][k] = Jxb[gix(mp, B, ex, ey, i, j)] / (mp.J * twg[i] * wy);
      }
      {
        const int i = k % A, j = k / A;
        const double wx = (i == 0 || i == A - 1) ? tww[0] + tww[A - 1] : tww[i];
        ly[el][k] = Jyb[gix(mp, B, ex, ey, i, j)] / (mp.J * wx * twg[j]);
      }
    }
  }
  __syncthreads();
  if (act && t < AA) {  // B_x-bar and B_y-bar at the (m+2)^2 Gauss points
    const int qx = t % A, qy = t / A;
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < A; ++j)
      for (int i = 0; i < A; ++i) {
        sx += lz[el][j * A + i] * tIWQ[qx][i] * tDWQ[qy][j];
        sy += lz[el][j * A + i] * tDWQ[qx][i] * tIWQ[qy][j];
      }
    const double wgt = mp.J * twq[qx] * twq[qy];
    qx_[el][t] = wgt * (2.0 / mp.hy) * sx;
    qy_[el][t] = -wgt * (2.0 / mp.hx) * sy;
  }
  if (act && t < BB) {  // B_z-bar at the Gauss_m points (gx, gy)
    const int gx = t % B, gy = t / B;
    double s = 0.0;
    for (int j = 0; j < A; ++j) s += -(2.0 / mp.hy) * mp.J * twg[gx] * twg[gy] * tDWG[gy][j] * lx[el][j * B + gx];
    for (int i = 0; i < A; ++i) s += (2.0 / mp.hx) * mp.J * twg[gy] * twg[gx] * tDWG[gx][i] * ly[el][gy * A + i];
    zg[el][t] = s;
  }
  __syncthreads();
  if (!act) return;
  double* BLe = BL + e * (2 * AB + BB);
  if (t < AB) {
    {  // B_x local (i < A, j < B): B_x(q) = sum I_G_Q[qy][j] I_W_Q[qx][i] bx
      const int i = t % A, j = t / A;
      double s = 0.0;
      for (int qy = 0; qy < A; ++qy)
        for (int qx = 0; qx < A; ++qx) s += tIGQ[qy][j] * tIWQ[qx][i] * qx_[el][qy * A + qx];
      BLe[t] += s;
    }
    {  // B_y local (i < B, j < A): B_y(q) = sum I_W_Q[qy][j] I_G_Q[qx][i] by
      const int i = t % B, j = t / B;
      double s = 0.0;
      for (int qy = 0; qy < A; ++qy)
        for (int qx = 0; qx < A; ++qx) s += tIWQ[qy][j] * tIGQ[qx][i] * qy_[el][qy * A + qx];
      BLe[AB + t] += s;
    }
  }
  if (t < BB) {
    const int ii = t % B, jj = t / B;
    double s = 0.0;
    for (int gy = 0; gy < B; ++gy)
      for (int gx = 0; gx < B; ++gx) s += tIVG[gx][ii] * tIVG[gy][jj] * zg[el][gy * B + gx];
    BLe[2 * AB + t] += s;
  }
}

}  // namespace

// sum of per-element locals at shared nodes (no division): Nx layout (shared in y), Ny layout
// (shared in x), W layout (shared in both); outputs three grids.
template <int M>
__global__ __launch_bounds__(256) void k_gather_sum(const double* __restrict__ Lnx, const double* __restrict__ Lny,
                                                    const double* __restrict__ Lw, long stride, double* __restrict__ Onx,
                                                    double* __restrict__ Ony, double* __restrict__ Ow, MeshP mp) {
  constexpr int A = M + 2, B = M + 1;
  const long NX = (long)mp.nx * B, G = NX * mp.ny * B;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const long gy = row_of(mp, g / B), gx = g - gy * NX;  // g / (nx B) = (g / B) / nx
  const long ex = gx / B, ey = gy / B;
  const int i = gx - ex * B, j = gy - ey * B;
  auto wr = [](long a, long n) { return a < 0 ? a + n : a; };
  const long e = ey * mp.nx + ex;
  const long eL = ey * mp.nx + wr(ex - 1, mp.nx), eD = wr(ey - 1, mp.ny) * mp.nx + ex;
  const long eLD = wr(ey - 1, mp.ny) * mp.nx + wr(ex - 1, mp.nx);
  if (Ow) {
    double s = Lw[e * stride + j * A + i];
    if (i == 0) s += Lw[eL * stride + j * A + (A - 1)];
    if (j == 0) s += Lw[eD * stride + (A - 1) * A + i];
    if (i == 0 && j == 0) s += Lw[eLD * stride + (A - 1) * A + (A - 1)];
    Ow[g] = s;
  }
  if (Onx) {
    double s = Lnx[e * stride + j * B + i];
    if (j == 0) s += Lnx[eD * stride + (A - 1) * B + i];
    Onx[g] = s;
  }
  if (Ony) {
    double s = Lny[e * stride + j * A + i];
    if (i == 0) s += Lny[eL * stride + j * A + (A - 1)];
    Ony[g] = s;
  }
}

// B_z locals are element-owned: copy into the grid
template <int M>
__global__ void k_scatter_bz(const double* __restrict__ BL, long stride, long off, double* __restrict__ Oz, MeshP mp) {
  constexpr int B = M + 1;
  const long NX = (long)mp.nx * B, G = NX * mp.ny * B;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const long gy = row_of(mp, g / B), gx = g - gy * NX;  // g / (nx B) = (g / B) / nx
  const long ex = gx / B, ey = gy / B;
  const int i = gx - ex * B, j = gy - ey * B;
  Oz[g] = BL[(ey * mp.nx + ex) * stride + off + j * B + i];
}

// ---------------------------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------------------------
#define DISPATCH_PV(p, F) \
  switch (p) { case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; \
               case 4: F(4); break; case 5: F(5); break; case 6: F(6); break; default: return -4; }
#define DISPATCH_PMV(p, m, F)                                                                             \
  if (p == 1 && m == 0) { F(1, 0); } else if (p == 1 && m == 1) { F(1, 1); }                              \
  else if (p == 2 && m == 1) { F(2, 1); } else if (p == 2 && m == 2) { F(2, 2); }                         \
  else if (p == 3 && m == 2) { F(3, 2); } else if (p == 3 && m == 3) { F(3, 3); }                         \
  else if (p == 4 && m == 3) { F(4, 3); } else if (p == 4 && m == 4) { F(4, 4); }                         \
  else if (p == 5 && m == 4) { F(5, 4); } else if (p == 5 && m == 5) { F(5, 5); }                         \
  else if (p == 6 && m == 5) { F(6, 5); } else if (p == 6 && m == 6) { F(6, 6); }                         \
  else return -4;
#define DISPATCH_MV(m, F) \
  switch (m) { case 0: F(0); break; case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; \
               case 4: F(4); break; case 5: F(5); break; case 6: F(6); break; default: return -4; }

int mag_reconstruct_JE(mhd25_ctx* c, const double* u, const double* Bx, const double* By, const double* Bz,
                       const double* eta, double* JE, bool r2);

static int vchk(mhd25_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { c->err = std::string(what) + ": " + hipGetErrorString(e); return -2; }
  return 0;
}

extern "C" int mhd25_rhs_hydro_vjp(mhd25_ctx* c, const double* U, const double* cot, double* Ubar) {
  if (!c || !U || !cot || !Ubar) return -1;
  const int eb = 256 / c->nn;
  const long blocks = (c->mp.K + eb - 1) / eb;
#define HV(P) hipLaunchKernelGGL((k_hydro_vjp<P>), dim3(blocks), dim3(256), 0, c->stream, U, cot, Ubar, c->d_ht, c->mp, \
                                 c->opt.iface_flux)
  DISPATCH_PV(c->p, HV);
#undef HV
  return vchk(c, "hydro vjp launch");
}

extern "C" int mhd25_rhs_magnetic_vjp(mhd25_ctx* c, const double* rho, const double* u, const double* Bx,
                                      const double* By, const double* Bz, const double* eta, const double* de_c,
                                      const double* du_c, const double* dBx_c, const double* dBy_c,
                                      const double* dBz_c, double* ubar, double* Bxb, double* Byb, double* Bzb) {
  if (!c || !rho || !u || !Bx || !By || !Bz || !de_c || !du_c || !dBx_c || !dBy_c || !dBz_c || !ubar || !Bxb ||
      !Byb || !Bzb)
    return -1;
  const long K = c->mp.K, G = c->G;
  const int a = c->m + 2, b = c->m + 1;
  const long loc = 2L * a * b + (long)a * a, bloc = 2L * a * b + (long)b * b;
  if (!c->vjp_scratch) {
    hipError_t e = hipMalloc((void**)&c->vjp_scratch, (size_t)K * (2 * loc + bloc) * 8 + 3 * G * 8 * 2);
    if (e != hipSuccess) { c->err = "vjp scratch allocation failed"; return -3; }
  }
  double* EL = c->vjp_scratch;
  double* JL = EL + K * loc;
  double* BL = JL + K * loc;
  double* Ebar = BL + K * bloc;  // 3G
  double* Jbar = Ebar + 3 * G;   // 3G
  // forward recomputation of J and E
  int r = mag_reconstruct_JE(c, u, Bx, By, Bz, eta, c->JE, false);  // the VJP reads every grid
  if (r) return r;
  int nn = (c->p + 1) * (c->p + 1), aa = a * a;
  const int eb = 256 / (nn > aa ? nn : aa);
  const long nb = (K + eb - 1) / eb;
  const long gb = (G + 255) / 256;
#define VU(P, M) hipLaunchKernelGGL((k_vjp_update<P, M>), dim3(nb), dim3(256), 0, c->stream, rho, Bx, By, Bz, c->JE, eta, \
                                    de_c, du_c, dBx_c, dBy_c, dBz_c, EL, JL, BL, c->d_mt, c->mp, G)
  DISPATCH_PMV(c->p, c->m, VU);
#undef VU
  // E-bar grids (sum of the curl-transpose locals)
#define GS(M) hipLaunchKernelGGL((k_gather_sum<M>), dim3(gb), dim3(256), 0, c->stream, EL, EL + a * b, EL + 2 * a * b, \
                                 loc, Ebar, Ebar + G, Ebar + 2 * G, c->mp)
  DISPATCH_MV(c->m, GS);
#undef GS
#define VE(P, M) hipLaunchKernelGGL((k_vjp_E<P, M>), dim3(nb), dim3(256), 0, c->stream, u, Bx, By, Bz, Ebar, eta, ubar, JL, \
                                    BL, c->d_mt, c->mp, G)
  DISPATCH_PMV(c->p, c->m, VE);
#undef VE
#define GJ(M) hipLaunchKernelGGL((k_gather_sum<M>), dim3(gb), dim3(256), 0, c->stream, JL, JL + a * b, JL + 2 * a * b, \
                                 loc, Jbar, Jbar + G, Jbar + 2 * G, c->mp)
  DISPATCH_MV(c->m, GJ);
#undef GJ
#define VJ(P, M) hipLaunchKernelGGL((k_vjp_J<P, M>), dim3(nb), dim3(256), 0, c->stream, Jbar, BL, c->d_mt, c->mp, G)
  DISPATCH_PMV(c->p, c->m, VJ);
#undef VJ
  // B-bar: B_x locals have the Ny layout, B_y locals the Nx layout, B_z element-owned
#define GB(M) hipLaunchKernelGGL((k_gather_sum<M>), dim3(gb), dim3(256), 0, c->stream, BL + a * b, BL, (const double*)nullptr, \
                                 bloc, Byb, Bxb, (double*)nullptr, c->mp)
  DISPATCH_MV(c->m, GB);
#undef GB
#define SZ(M) hipLaunchKernelGGL((k_scatter_bz<M>), dim3(gb), dim3(256), 0, c->stream, BL, bloc, 2L * a * b, Bzb, c->mp)
  DISPATCH_MV(c->m, SZ);
#undef SZ
  return vchk(c, "magnetic vjp launch");
}
