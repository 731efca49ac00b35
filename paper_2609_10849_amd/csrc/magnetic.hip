// Magnetic-velocity subflow kernels for gfx950 (section "Magnetic--velocity subflow:
// compatible finite elements").
//
// Element-local kernels use one block per tile of EB elements and NT = max((p+1)^2,(m+2)^2)
// threads per element; element data are staged in LDS.  Loads of shared degrees of freedom
// are written per element and summed by a per-node gather in a fixed order (no floating-point
// atomics), then divided by the lumped weights (eq. quad-hcurl-element, eq. quad-cg-element).
#include <cfloat>
#include <mutex>
#include <string>

#include "common.h"
#include "xcd.h"
#include "rsqrt.h"

namespace {

constexpr double EPSM = 2.220446049250313e-16;

template <int P, int M, int BS = 256>
struct MC {
  static constexpr int NP = P + 1, NN = NP * NP, A = M + 2, B = M + 1, AA = A * A, AB = A * B, BB = B * B;
  static constexpr int NT = NN > AA ? NN : AA;
  static constexpr int EB = BS / NT;
};

__device__ __forceinline__ long wrapl(long a, long n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// global index of local node (i, j) of element (ex, ey) on a magnetic grid (32-bit arithmetic: a
// grid holds fewer than 2^29 nodes, which mhd25_init guarantees)
__device__ __forceinline__ long gix(const MeshP& mp, int B, long ex, long ey, int i, int j) {
  const int NX = mp.nx * B, NY = mp.ny * B;
  int gx = (int)ex * B + i, gy = (int)ey * B + j;
  if (gx >= NX) gx -= NX;
  if (gy >= NY) gy -= NY;
  return (long)(gy * NX + gx);
}

// R2: the 2D2V reduced system (u_z = B_z = 0, in-plane E and J identically zero); B_z is not read
template <int P, int M, bool R2 = false>
__device__ __forceinline__ void load_B(double* bx, double* by, double* bz, const double* __restrict__ Bx,
                                       const double* __restrict__ By, const double* __restrict__ Bz, const MeshP& mp,
                                       long ex, long ey, int t) {
  using C = MC<P, M>;
  for (int k = t; k < C::AB; k += C::NT) {
    bx[k] = Bx[gix(mp, C::B, ex, ey, k % C::A, k / C::A)];  // [j<B][i<A]
    by[k] = By[gix(mp, C::B, ex, ey, k % C::B, k / C::B)];  // [j<A][i<B]
  }
  if constexpr (!R2)
    for (int k = t; k < C::BB; k += C::NT) bz[k] = Bz[gix(mp, C::B, ex, ey, k % C::B, k / C::B)];
}

// ---------------------------------------------------------------------------------------------
// Current loads (eq. mag-current-proj): W part int B_x d_y phi - B_y d_x phi with the (m+2)-point
// Gauss rule; N parts int B_z (-d_y psi) and int B_z d_x psi with the (m+1)-point rule.
// ---------------------------------------------------------------------------------------------
template <int P, int M, int BS, bool R2>
__device__ __forceinline__ void J_loads_body(const double* __restrict__ Bx, const double* __restrict__ By,
                                                 const double* __restrict__ Bz, double* __restrict__ Lx,
                                                 double* __restrict__ Ly, double* __restrict__ Lz,
                                                 const MagTab* __restrict__ T, MeshP mp, long blk) {
  using C = MC<P, M, BS>;
  constexpr int A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB, NT = C::NT;
  __shared__ double sbx[EB][AB], sby[EB][AB], sbz[EB][BB], swx[EB][AA], swy[EB][AA], szg[EB][BB];
  __shared__ double sh[EB][2][AA];  // first half of the sum factorisation of the W loads
  __shared__ double tWQ[A][A], tGQ[A][B], tDWQ[A][A], tVG[B][B], tDWG[B][A], twq[A], twg[B];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  const long e = blk * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  for (int k = tid; k < A * A; k += BS) {
    tWQ[k / A][k % A] = T->I_W_Q[k / A][k % A];
    tDWQ[k / A][k % A] = T->D_W_Q[k / A][k % A];
  }
  for (int k = tid; k < A * B; k += BS) tGQ[k / B][k % B] = T->I_G_Q[k / B][k % B];
  for (int k = tid; k < B * B; k += BS) tVG[k / B][k % B] = T->I_V_G[k / B][k % B];
  for (int k = tid; k < B * A; k += BS) tDWG[k / A][k % A] = T->D_W_G[k / A][k % A];
  if (tid < A) twq[tid] = T->wq[tid];
  if (tid < B) twg[tid] = T->wg[tid];
  if (act) load_B<P, M, R2>(sbx[el], sby[el], sbz[el], Bx, By, Bz, mp, ex, ey, t);
  __syncthreads();
  if (act && t < AA) {
    const int qx = t % A, qy = t / A;
    double bxq = 0.0, byq = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) s += tWQ[qx][i] * sbx[el][j * A + i];
      bxq += tGQ[qy][j] * s;
    }
#pragma unroll
    for (int j = 0; j < A; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tGQ[qx][i] * sby[el][j * B + i];
      byq += tWQ[qy][j] * s;
    }
    const double wgt = mp.J * twq[qx] * twq[qy];
    swx[el][t] = wgt * bxq;
    swy[el][t] = wgt * byq;
  }
  if (!R2 && act && t < BB) {  // B_z at the Gauss nodes (the N loads; none in the 2D2V system)
    const int gx = t % B, gy = t / B;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tVG[gx][i] * sbz[el][j * B + i];
      v += tVG[gy][j] * s;
    }
    szg[el][t] = v;
  }
  __syncthreads();
  // W loads, factorised: sh[0][qy][i] = sum_qx I_W_Q[qx][i] swx[qy][qx], sh[1][qy][i] = sum_qx D_W_Q[qx][i] swy[qy][qx]
  if (act && t < AA) {
    const int i = t % A, qy = t / A;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int qx = 0; qx < A; ++qx) {
      a0 += tWQ[qx][i] * swx[el][qy * A + qx];
      a1 += tDWQ[qx][i] * swy[el][qy * A + qx];
    }
    sh[el][0][t] = a0;
    sh[el][1][t] = a1;
  }
  __syncthreads();
  if (!act) return;
  if (t < AA) {
    const int i = t % A, j = t / A;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int qy = 0; qy < A; ++qy) {
      sx += tDWQ[qy][j] * sh[el][0][qy * A + i];
      sy += tWQ[qy][j] * sh[el][1][qy * A + i];
    }
    Lz[e * AA + t] = (2.0 * mp.rhy) * sx - (2.0 * mp.rhx) * sy;
  }
  if (!R2 && t < AB) {
    {  // N_x node: i Gauss (B), j GLL (A); index j*B + i
      const int i = t % B, j = t / B;
      double s = 0.0;
#pragma unroll
      for (int qy = 0; qy < B; ++qy) s += twg[qy] * szg[el][qy * B + i] * tDWG[qy][j];
      Lx[e * AB + t] = -(2.0 * mp.rhy) * mp.J * twg[i] * s;
    }
    {  // N_y node: i GLL (A), j Gauss (B); index j*A + i
      const int i = t % A, j = t / A;
      double s = 0.0;
#pragma unroll
      for (int qx = 0; qx < B; ++qx) s += twg[qx] * szg[el][j * B + qx] * tDWG[qx][i];
      Ly[e * AB + t] = (2.0 * mp.rhx) * mp.J * twg[j] * s;
    }
  }
}

template <int P, int M, int BS, bool R2>
__global__ __launch_bounds__(BS) void k_J_loads(const double* __restrict__ Bx, const double* __restrict__ By,
                                                 const double* __restrict__ Bz, double* __restrict__ Lx,
                                                 double* __restrict__ Ly, double* __restrict__ Lz,
                                                 const MagTab* __restrict__ T, MeshP mp) {
  J_loads_body<P, M, BS, R2>(Bx, By, Bz, Lx, Ly, Lz, T, mp, xcd_block());
}

struct J_loads_args {
  const double* Bx;
  const double* By;
  const double* Bz;
  double* Lx;
  double* Ly;
  double* Lz;
  const MagTab* T;
  MeshP mp;
};

template <int P, int M, int BS, bool R2>
__global__ __launch_bounds__(BS) void k_J_loads_rt(const J_loads_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const J_loads_args& a = A[r];
  J_loads_body<P, M, BS, R2>(gl(a.Bx), gl(a.By), gl(a.Bz), gl(a.Lx), gl(a.Ly), gl(a.Lz), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

// ---------------------------------------------------------------------------------------------
// Electric-field loads (eq. mag-electric-proj): w_a (-u x B)|_K at the element's own auxiliary
// nodes, plus eta_K sum_q M_q J(x_q) . phi_a(x_q) by the degree-p GLL rule.
// ---------------------------------------------------------------------------------------------
template <int P, int M, int BS, bool R2>
__device__ __forceinline__ void E_loads_body(const double* __restrict__ u, const double* __restrict__ Bx,
                                                 const double* __restrict__ By, const double* __restrict__ Bz,
                                                 const double* __restrict__ Jx, const double* __restrict__ Jy,
                                                 const double* __restrict__ Jz, const double* __restrict__ eta,
                                                 double* __restrict__ Lx, double* __restrict__ Ly,
                                                 double* __restrict__ Lz, const MagTab* __restrict__ T, MeshP mp, long blk) {
  using C = MC<P, M, BS>;
  constexpr int NP = C::NP, NN = C::NN, A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB,
                NT = C::NT;
  // J on the auxiliary grids (sjx, sjy, sjz), and later the x sums of the eta term (sxj)
  constexpr int NJ = 2 * AB + AA, NXJ = NP * (B + 2 * A), NJB = NJ > NXJ ? NJ : NXJ;
  __shared__ double su[EB][3][NN], sbx[EB][AB], sby[EB][AB], sbz[EB][BB];
  __shared__ double sjb[EB][NJB];
  // the eta-weighted J values at the GLL_p nodes reuse su once the x interpolation has read it
  // (with 96 VGPRs and 14.8 KB of LDS per 128-thread block at N = 4: 5 waves per SIMD)
  double(*const swj)[3][NN] = su;
  __shared__ double sux[EB][3][NP][A + B];  // velocity interpolated in x: [d][qj][W nodes | Gauss nodes]
  __shared__ double tGP[NP][B], tWP[NP][A], tPW[A][NP], tPG[B][NP], tGW[A][B], tVG[B][B], tVW[A][B];
  __shared__ double twp[NP], tww[A], twg[B];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  const long e = blk * EB + el;
  const bool act = el < EB && e < mp.K;
  double* const sjx = sjb[el < EB ? el : 0];  // [j < A][i < B]
  double* const sjy = sjx + AB;                // [j < B][i < A]
  double* const sjz = sjx + 2 * AB;            // [j < A][i < A]
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  const double et = (act && eta) ? eta[e] : 0.0;
  for (int k = tid; k < NP * B; k += BS) tGP[k / B][k % B] = T->I_G_P[k / B][k % B];
  for (int k = tid; k < NP * A; k += BS) {
    tWP[k / A][k % A] = T->I_W_P[k / A][k % A];
    tPW[k / NP][k % NP] = T->I_P_W[k / NP][k % NP];
  }
  for (int k = tid; k < B * NP; k += BS) tPG[k / NP][k % NP] = T->I_P_G[k / NP][k % NP];
  for (int k = tid; k < A * B; k += BS) {
    tGW[k / B][k % B] = T->I_G_W[k / B][k % B];
    tVW[k / B][k % B] = T->I_V_W[k / B][k % B];
  }
  for (int k = tid; k < B * B; k += BS) tVG[k / B][k % B] = T->I_V_G[k / B][k % B];
  if (tid < NP) twp[tid] = T->wp[tid];
  if (tid < A) tww[tid] = T->ww[tid];
  if (tid < B) twg[tid] = T->wg[tid];
  constexpr int NU = R2 ? 2 : 3;  // velocity components carried (u_z = 0 in the 2D2V system)
  if (act) {
    for (int k = t; k < NN; k += NT)
      for (int d = 0; d < NU; ++d) su[el][d][k] = u[d * KN + e * NN + k];
    load_B<P, M, R2>(sbx[el], sby[el], sbz[el], Bx, By, Bz, mp, ex, ey, t);
    if (et != 0.0) {
      if constexpr (!R2)
        for (int k = t; k < AB; k += NT) {
          sjx[k] = Jx[gix(mp, B, ex, ey, k % B, k / B)];
          sjy[k] = Jy[gix(mp, B, ex, ey, k % A, k / A)];
        }
      for (int k = t; k < AA; k += NT) sjz[k] = Jz[gix(mp, B, ex, ey, k % A, k / A)];
    }
  }
  __syncthreads();
  if (act) {
    // first half of the sum factorisation of u at the auxiliary nodes: interpolate in x
    // (the 2D2V system needs u_x, u_y at the W nodes only: x < A)
    constexpr int NX = R2 ? A : A + B;
    for (int tk = t; tk < NU * NP * NX; tk += NT) {
      const int d = tk / (NP * NX), rem = tk - d * NP * NX, qj = rem / NX, x = rem - qj * NX;
      const double* I = x < A ? tPW[x] : tPG[x - A];
      double v = 0.0;
#pragma unroll
      for (int qi = 0; qi < NP; ++qi) v += I[qi] * su[el][d][qj * NP + qi];
      sux[el][d][qj][x] = v;
    }
  }
  const bool jnode = act && et != 0.0 && t < NN;
  double jw[3] = {0.0, 0.0, 0.0};
  if (jnode) {
    const int qi = t % NP, qj = t / NP;
    double jx = 0.0, jy = 0.0, jz = 0.0;
    if constexpr (!R2) {
#pragma unroll
      for (int j = 0; j < A; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < B; ++i) s += tGP[qi][i] * sjx[j * B + i];
        jx += tWP[qj][j] * s;
      }
#pragma unroll
      for (int j = 0; j < B; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < A; ++i) s += tWP[qi][i] * sjy[j * A + i];
        jy += tGP[qj][j] * s;
      }
    }
#pragma unroll
    for (int j = 0; j < A; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) s += tWP[qi][i] * sjz[j * A + i];
      jz += tWP[qj][j] * s;
    }
    const double w = et * mp.J * twp[qi] * twp[qj];
    jw[0] = w * jx; jw[1] = w * jy; jw[2] = w * jz;
  }
  __syncthreads();  // every lane has finished reading su and the J grids
  if (jnode) { swj[el][0][t] = jw[0]; swj[el][1][t] = jw[1]; swj[el][2][t] = jw[2]; }
  __syncthreads();
  // the eta term sum_q M_q (eta J)(x_q) phi_a(x_q) by sum factorisation: x sums first, into the
  // J-grid space, xs0[qj][i < B] (G in x, for E_x), xs1[qj][i < A] and xs2[qj][i < A] (W in x)
  double* const xs0 = sjx;
  double* const xs1 = xs0 + NP * B;
  double* const xs2 = xs1 + NP * A;
  if (act && et != 0.0) {
    for (int tk = t; tk < NXJ; tk += NT) {
      int c, qj, i;
      if (tk < NP * B) { c = 0; qj = tk / B; i = tk - qj * B; }
      else { const int r = (tk - NP * B) % (NP * A); c = 1 + (tk - NP * B) / (NP * A); qj = r / A; i = r - qj * A; }
      if (R2 && c < 2) continue;
      double v = 0.0;
#pragma unroll
      for (int qi = 0; qi < NP; ++qi) v += (c == 0 ? tGP[qi][i] : tWP[qi][i]) * swj[el][c][qj * NP + qi];
      xs0[tk] = v;
    }
  }
  __syncthreads();
  if (!act) return;
  // second half: interpolate in y (Iy = I_P_W or I_P_G row aj; x column xc of sux)
  auto u_at = [&](int d, const double* Iy, int xc) {
    double v = 0.0;
#pragma unroll
    for (int qj = 0; qj < NP; ++qj) v += Iy[qj] * sux[el][d][qj][xc];
    return v;
  };
  // y sums of the eta term: xs[qj * nx + ai] against the y basis column aj
  auto eta_term = [&](const double* xs, int nx, int ai, bool ygauss, int aj) {
    double v = 0.0;
#pragma unroll
    for (int qj = 0; qj < NP; ++qj) v += (ygauss ? tGP[qj][aj] : tWP[qj][aj]) * xs[qj * nx + ai];
    return v;
  };
  if (t < AA) {  // W node (xw[i], xw[j]): z-component
    const int i = t % A, j = t / A;
    const double ux = u_at(0, tPW[j], i), uy = u_at(1, tPW[j], i);
    double bxv = 0.0, byv = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      bxv += tGW[j][k] * sbx[el][k * A + i];
      byv += tGW[i][k] * sby[el][j * B + k];
    }
    double s = mp.J * tww[i] * tww[j] * (-(ux * byv - uy * bxv));
    if (et != 0.0) s += eta_term(xs2, A, i, false, j);
    Lz[e * AA + t] = s;
  }
  if (!R2 && t < AB) {
    {  // N_x node (xg[i], xw[j]): x-component; B_y lives on these nodes
      const int i = t % B, j = t / B;
      const double uy = u_at(1, tPW[j], A + i), uz = u_at(2, tPW[j], A + i);
      const double byv = sby[el][t];
      double bzv = 0.0;
#pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < B; ++ii) s += tVG[i][ii] * sbz[el][jj * B + ii];
        bzv += tVW[j][jj] * s;
      }
      double s = mp.J * twg[i] * tww[j] * (-(uy * bzv - uz * byv));
      if (et != 0.0) s += eta_term(xs0, B, i, false, j);
      Lx[e * AB + t] = s;
    }
    {  // N_y node (xw[i], xg[j]): y-component; B_x lives on these nodes
      const int i = t % A, j = t / A;
      const double ux = u_at(0, tPG[j], i), uz = u_at(2, tPG[j], i);
      const double bxv = sbx[el][t];
      double bzv = 0.0;
#pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < B; ++ii) s += tVW[i][ii] * sbz[el][jj * B + ii];
        bzv += tVG[j][jj] * s;
      }
      double s = mp.J * tww[i] * twg[j] * (-(uz * bxv - ux * bzv));
      if (et != 0.0) s += eta_term(xs1, A, i, true, j);
      Ly[e * AB + t] = s;
    }
  }
}

template <int P, int M, int BS, bool R2>
__global__ __launch_bounds__(BS, (!R2 && P <= 5) ? 5 : 1) void k_E_loads(const double* __restrict__ u, const double* __restrict__ Bx,
                                                 const double* __restrict__ By, const double* __restrict__ Bz,
                                                 const double* __restrict__ Jx, const double* __restrict__ Jy,
                                                 const double* __restrict__ Jz, const double* __restrict__ eta,
                                                 double* __restrict__ Lx, double* __restrict__ Ly,
                                                 double* __restrict__ Lz, const MagTab* __restrict__ T, MeshP mp) {
  E_loads_body<P, M, BS, R2>(u, Bx, By, Bz, Jx, Jy, Jz, eta, Lx, Ly, Lz, T, mp, xcd_block());
}

struct E_loads_args {
  const double* u;
  const double* Bx;
  const double* By;
  const double* Bz;
  const double* Jx;
  const double* Jy;
  const double* Jz;
  const double* eta;
  double* Lx;
  double* Ly;
  double* Lz;
  const MagTab* T;
  MeshP mp;
};

template <int P, int M, int BS, bool R2>
__global__ __launch_bounds__(BS, (!R2 && P <= 5) ? 5 : 1) void k_E_loads_rt(const E_loads_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const E_loads_args& a = A[r];
  E_loads_body<P, M, BS, R2>(gl(a.u), gl(a.Bx), gl(a.By), gl(a.Bz), gl(a.Jx), gl(a.Jy), gl(a.Jz), gl(a.eta), gl(a.Lx), gl(a.Ly), gl(a.Lz), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

// ---------------------------------------------------------------------------------------------
// Curl update, Lorentz transpose and Ohmic heating (eq. magnetic-dae with J, E eliminated).
// MODE 0: write L_M.  MODE 1: write the SSP stage (ca*Y^n + cb*Y_s) + cb*tau*L_M(Y_s).
// ---------------------------------------------------------------------------------------------

// (the 2D2V variants up to N = 4 fit 72 VGPRs, i.e. 7 waves per SIMD, without spills; the bound
// keeps the compiler there)
template <int P, int M, int MODE, int BS, bool R2>
__device__ __forceinline__ void mag_update_body(MagIO io, const MagTab* __restrict__ T, MeshP mp, long blk) {
  using C = MC<P, M, BS>;
  constexpr int NP = C::NP, NN = C::NN, A = C::A, B = C::B, AA = C::AA, AB = C::AB, BB = C::BB, EB = C::EB,
                NT = C::NT;
  __shared__ double sbx[EB][AB], sby[EB][AB], sbz[EB][BB];
  __shared__ double sex[EB][AB], sey[EB][AB], sez[EB][AA];
  __shared__ double sjx[EB][AB], sjy[EB][AB], sjz[EB][AA];
  // Lorentz loads at the auxiliary nodes, one buffer per element: fz (W nodes, x and y parts), fx
  // (N_x nodes, y and z parts), fy (N_y nodes, x and z parts).  After a barrier the new velocities
  // for the closing element statistics reuse it, which keeps the block's LDS within five blocks
  // per CU at N = 4.
  constexpr int NF = 2 * AA + 4 * AB;
  static_assert(3 * NN <= NF, "the velocity buffer must fit in the Lorentz-load buffer");
  __shared__ double sf[EB][NF];
  __shared__ double tDWG[B][A], tDWV[B][A], tIGV[B][B], tIGW[A][B], tIVG[B][B], tIVW[A][B], tIPW[A][NP], tIPG[B][NP], tIGP[NP][B], tIWP[NP][A];
  __shared__ double tww[A], twg[B], twp[NP];
  const int tid = threadIdx.x, el = tid / NT, t = tid - el * NT;
  const long e = blk * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  double* const fz = sf[act ? el : 0];
  double* const fx = fz + 2 * AA;
  double* const fy = fx + 2 * AB;
  for (int k = tid; k < B * A; k += BS) tDWG[k / A][k % A] = T->D_W_G[k / A][k % A];
  for (int k = tid; k < B * A; k += BS) tDWV[k / A][k % A] = T->D_W_V[k / A][k % A];
  for (int k = tid; k < B * B; k += BS) tIGV[k / B][k % B] = T->I_G_V[k / B][k % B];
  for (int k = tid; k < A * B; k += BS) tIGW[k / B][k % B] = T->I_G_W[k / B][k % B];
  for (int k = tid; k < B * B; k += BS) tIVG[k / B][k % B] = T->I_V_G[k / B][k % B];
  for (int k = tid; k < A * B; k += BS) tIVW[k / B][k % B] = T->I_V_W[k / B][k % B];
  for (int k = tid; k < A * NP; k += BS) tIPW[k / NP][k % NP] = T->I_P_W[k / NP][k % NP];
  for (int k = tid; k < B * NP; k += BS) tIPG[k / NP][k % NP] = T->I_P_G[k / NP][k % NP];
  for (int k = tid; k < NP * B; k += BS) tIGP[k / B][k % B] = T->I_G_P[k / B][k % B];
  for (int k = tid; k < NP * A; k += BS) tIWP[k / A][k % A] = T->I_W_P[k / A][k % A];
  if (tid < A) tww[tid] = T->ww[tid];
  if (tid < B) twg[tid] = T->wg[tid];
  if (tid < NP) twp[tid] = T->wp[tid];
  // values used only at the end are loaded first, so that their latency overlaps the work
  // (MODE 1 keeps only y0 = ca*Y^n + cb*Y_s of every value and adds cb*tau*L_M at the end, so
  // that one register pair per value stays live across the kernel instead of two)
  double rq = 1.0, et = 0.0, y0[4] = {0, 0, 0, 0}, b0[3] = {0, 0, 0};
  long gown = 0;
  if (act && t < NN) {
    const long n = e * NN + t;
    rq = io.rho[n];
    et = io.eta ? io.eta[e] : 0.0;
    if (MODE == 1) {
#pragma unroll
      for (int d = 0; d < (R2 ? 2 : 3); ++d) y0[d] = io.ca * io.un[d * KN + n] + io.cb * io.us[d * KN + n];
      y0[3] = io.ca * io.en[n] + io.cb * io.es[n];
    }
  }
  if (act && t < BB) {
    gown = gix(mp, B, ex, ey, t % B, t / B);
    if (MODE == 1) {
      b0[0] = io.ca * io.bxn[gown] + io.cb * io.bxs[gown];
      b0[1] = io.ca * io.byn[gown] + io.cb * io.bys[gown];
      if (!R2) b0[2] = io.ca * io.bzn[gown] + io.cb * io.bzs[gown];
    }
  }
  if (act) {
    load_B<P, M, R2>(sbx[el], sby[el], sbz[el], io.bxs, io.bys, io.bzs, mp, ex, ey, t);
    for (int k = t; !R2 && k < AB; k += NT) {  // in-plane E and J (none in the 2D2V system)
      const long gN_x = gix(mp, B, ex, ey, k % B, k / B), gN_y = gix(mp, B, ex, ey, k % A, k / A);
      sex[el][k] = io.ex[gN_x]; sjx[el][k] = io.jx[gN_x];
      sey[el][k] = io.ey[gN_y]; sjy[el][k] = io.jy[gN_y];
    }
    for (int k = t; k < AA; k += NT) {
      const long g = gix(mp, B, ex, ey, k % A, k / A);
      sez[el][k] = io.ez[g]; sjz[el][k] = io.jz[g];
    }
  }
  __syncthreads();
  if (act && t < BB) {  // strong curl at the element's owned B nodes
    const int i = t % B, j = t / B;
    const long g = gown;
    double dbx = 0.0, dby = 0.0;
#pragma unroll
    for (int k = 0; k < A; ++k) {
      dbx += tDWG[j][k] * sez[el][k * A + i];
      dby += tDWG[i][k] * sez[el][j * A + k];
    }
    dbx *= -(2.0 * mp.rhy);
    dby *= (2.0 * mp.rhx);
    double dxey = 0.0, dyex = 0.0;
    if constexpr (!R2) {
#pragma unroll
    for (int l = 0; l < B; ++l) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < A; ++k) s += tDWV[i][k] * sey[el][l * A + k];
      dxey += tIGV[j][l] * s;
    }
#pragma unroll
    for (int l = 0; l < A; ++l) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) s += tIGV[i][k] * sex[el][l * B + k];
      dyex += tDWV[j][l] * s;
    }
    }
    const double dbz = R2 ? 0.0 : -((2.0 * mp.rhx) * dxey - (2.0 * mp.rhy) * dyex);
    if (MODE == 0) {
      io.obx[g] = dbx; io.oby[g] = dby; io.obz[g] = dbz;
    } else {
      const double ct = io.cb * io.tau;
      io.obx[g] = b0[0] + ct * dbx;
      io.oby[g] = b0[1] + ct * dby;
      io.obz[g] = R2 ? 0.0 : b0[2] + ct * dbz;
    }
  }
  // weighted Lorentz loads f_a at the auxiliary nodes (transpose of the coupling form)
  if (act && t < AA) {
    const int i = t % A, j = t / A;
    double bxv = 0.0, byv = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      bxv += tIGW[j][k] * sbx[el][k * A + i];
      byv += tIGW[i][k] * sby[el][j * B + k];
    }
    const double w = mp.J * tww[i] * tww[j] * sjz[el][t];
    fz[t] = -byv * w;      // x
    fz[AA + t] = bxv * w;  // y
  }
  if (!R2 && act && t < AB) {
    {
      const int i = t % B, j = t / B;  // N_x node: (0, -B_z J_x, B_y J_x)
      double bzv = 0.0;
#pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < B; ++ii) s += tIVG[i][ii] * sbz[el][jj * B + ii];
        bzv += tIVW[j][jj] * s;
      }
      const double w = mp.J * twg[i] * tww[j] * sjx[el][t];
      fx[t] = -bzv * w;             // y
      fx[AB + t] = sby[el][t] * w;  // z
    }
    {
      const int i = t % A, j = t / A;  // N_y node: (B_z J_y, 0, -B_x J_y)
      double bzv = 0.0;
#pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int ii = 0; ii < B; ++ii) s += tIVW[i][ii] * sbz[el][jj * B + ii];
        bzv += tIVG[j][jj] * s;
      }
      const double w = mp.J * tww[i] * twg[j] * sjy[el][t];
      fy[t] = bzv * w;               // x
      fy[AB + t] = -sbx[el][t] * w;  // z
    }
  }
  __syncthreads();
  const bool node = act && t < NN;
  double vnew[3] = {0.0, 0.0, 0.0};
  if (node) {
    const int qi = t % NP, qj = t / NP;
    // transpose of the interpolation to the auxiliary nodes, factorised over the two directions
    double du[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int j = 0; j < A; ++j) {
      double s0 = 0.0, s1 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) {
        const double I = tIPW[i][qi];
        s0 += I * fz[j * A + i];
        s1 += I * fz[AA + j * A + i];
      }
      if constexpr (!R2) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const double I = tIPG[i][qi];
          t1 += I * fx[j * B + i];
          t2 += I * fx[AB + j * B + i];
        }
      }
      const double Iy = tIPW[j][qj];
      du[0] += Iy * s0;
      du[1] += Iy * (s1 + t1);
      du[2] += Iy * t2;
    }
#pragma unroll 1
    for (int j = 0; !R2 && j < B; ++j) {
      double s0 = 0.0, s2 = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) {
        const double I = tIPW[i][qi];
        s0 += I * fy[j * A + i];
        s2 += I * fy[AB + j * A + i];
      }
      const double Iy = tIPG[j][qj];
      du[0] += Iy * s0;
      du[2] += Iy * s2;
    }
    const long n = e * NN + t;
    const double Mq = mp.J * twp[qi] * twp[qj];
    double de = 0.0;
    if (et != 0.0) {
      double jx = 0.0, jy = 0.0, jz = 0.0;
      if constexpr (!R2) {
#pragma unroll
        for (int j = 0; j < A; ++j) {
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < B; ++i) s += tIGP[qi][i] * sjx[el][j * B + i];
          jx += tIWP[qj][j] * s;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < A; ++i) s += tIWP[qi][i] * sjy[el][j * A + i];
          jy += tIGP[qj][j] * s;
        }
      }
#pragma unroll
      for (int j = 0; j < A; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < A; ++i) s += tIWP[qi][i] * sjz[el][j * A + i];
        jz += tIWP[qj][j] * s;
      }
      de = et * (jx * jx + jy * jy + jz * jz) * rcp_refined(rq);  // rho > 0
    }
    // (the 2D2V system writes u_z = 0, so that no stage buffer carries a stale value)
    const double irm = rcp_refined(rq * Mq);  // 1 / (rho M), both positive
    if (MODE == 0) {
      for (int d = 0; d < 3; ++d) io.ou[d * KN + n] = (R2 && d == 2) ? 0.0 : du[d] * irm;
      io.oe[n] = de;
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double v = (R2 && d == 2) ? 0.0 : y0[d] + (io.cb * io.tau) * (du[d] * irm);
        io.ou[d * KN + n] = v;
        vnew[d] = v;
      }
      io.oe[n] = y0[3] + (io.cb * io.tau) * de;
    }
  }
  if (MODE == 1 && io.ustats) {
    // element statistics of the new velocity (GLL-weighted sum, min, max), as the velocity-OE
    // sensor needs them
    __syncthreads();  // every lane has finished reading the Lorentz loads
    if (node)
#pragma unroll
      for (int d = 0; d < 3; ++d) fz[d * NN + t] = vnew[d];
    __syncthreads();
    constexpr int NU = R2 ? 2 : 3;  // statistics [K][NU][3] of the carried components
    for (int tk = t; act && tk < 3 * NU; tk += NT) {
      const int c = tk / 3, kind = tk - 3 * c;
      double sm = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
      for (int k = 0; k < NN; ++k) {
        const double v = fz[c * NN + k];
        sm += (twp[k % NP] * twp[k / NP]) * v;
        mn = fmin(mn, v); mx = fmax(mx, v);
      }
      io.ustats[(e * NU + c) * 3 + kind] = kind == 0 ? sm : (kind == 1 ? mn : mx);
    }
  }
}

template <int P, int M, int MODE, int BS, bool R2>
__global__ __launch_bounds__(BS, (R2 && P <= 4) ? 7 : 1) void k_mag_update(MagIO io, const MagTab* __restrict__ T, MeshP mp) {
  mag_update_body<P, M, MODE, BS, R2>(io, T, mp, xcd_block());
}

using ::gl;
// a MagIO read from a run-table argument struct, its pointers loaded as global-memory pointers
__device__ __forceinline__ MagIO gl(const MagIO& s) {
  MagIO o = s;
  o.rho = gl(s.rho); o.us = gl(s.us); o.es = gl(s.es); o.bxs = gl(s.bxs); o.bys = gl(s.bys); o.bzs = gl(s.bzs);
  o.un = gl(s.un); o.en = gl(s.en); o.bxn = gl(s.bxn); o.byn = gl(s.byn); o.bzn = gl(s.bzn);
  o.jx = gl(s.jx); o.jy = gl(s.jy); o.jz = gl(s.jz); o.ex = gl(s.ex); o.ey = gl(s.ey); o.ez = gl(s.ez);
  o.eta = gl(s.eta);
  o.oe = gl(s.oe); o.ou = gl(s.ou); o.obx = gl(s.obx); o.oby = gl(s.oby); o.obz = gl(s.obz);
  o.ustats = gl(s.ustats);
  return o;
}

struct mag_update_args {
  MagIO io;
  const MagTab* T;
  MeshP mp;
};

template <int P, int M, int MODE, int BS, bool R2>
__global__ __launch_bounds__(BS, (R2 && P <= 4) ? 7 : 1) void k_mag_update_rt(const mag_update_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const mag_update_args& a = A[r];
  mag_update_body<P, M, MODE, BS, R2>(gl(a.io), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

// per-element statistics of NC nodal fields [NC][K][NN] -> [K][NC][3] (GLL-weighted sum, min, max)
template <int P, int NC>
__global__ __launch_bounds__(256) void k_field_stats(const double* __restrict__ f, double* __restrict__ stats,
                                                     const MagTab* __restrict__ T, MeshP mp) {
  constexpr int NP = P + 1, NN = NP * NP, EB = 256 / NN;
  __shared__ double sv[NC][EB * NN];
  const int tid = threadIdx.x, el = tid / NN, q = tid - el * NN;
  const long e = (long)blockIdx.x * EB + el;
  const bool act = el < EB && e < mp.K;
  const long KN = mp.K * NN;
  if (act)
    for (int c = 0; c < NC; ++c) sv[c][tid] = f[c * KN + e * NN + q];
  __syncthreads();
  for (int tk = q; act && tk < NC * 3; tk += NN) {
    const int c = tk / 3, kind = tk - 3 * c;
    double s = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
    for (int k = 0; k < NN; ++k) {
      const double v = sv[c][el * NN + k];
      s += (T->wp[k % NP] * T->wp[k / NP]) * v;
      mn = fmin(mn, v); mx = fmax(mx, v);
    }
    stats[(e * NC + c) * 3 + kind] = kind == 0 ? s : (kind == 1 ? mn : mx);
  }
}

// ---------------------------------------------------------------------------------------------
// Velocity OE (eq. magnetic-oe-sensor .. eq. magnetic-oe-map).  The rho-weighted projections use
// the shell-ordered tensor Legendre basis orthonormalised in the rho-weighted product,
// psi = phi L^{-T} with G = L L^T the Gram matrix.  rho is frozen during a magnetic substep, so
// Psi[q][k] = psi_k(x_q) is computed once per substep (k_vel_prep) and reused by the three stages: per stage k_vel_sensor forms the
// damping factors and k_vel_proj applies the map.
// ---------------------------------------------------------------------------------------------
// shell index of mode k in the shell ordering (shell l holds modes l^2 .. (l+1)^2 - 1)
__host__ __device__ constexpr int shell_of(int k) {
  int l = 0;
  while ((l + 1) * (l + 1) <= k) ++l;
  return l;
}

// shell-ordered tensor Legendre mode k -> (a, b): shell l = max(a, b) holds modes l^2 .. (l+1)^2 - 1,
// (a, l) for a < l first, then (l, b) for b = 0..l (the order of the basis tables)
__host__ __device__ constexpr int mode_a(int k) {
  const int l = shell_of(k), r = k - l * l;
  return r < l ? r : l;
}
__host__ __device__ constexpr int mode_b(int k) {
  const int l = shell_of(k), r = k - l * l;
  return r < l ? l : r - l;
}

// threads per block of the velocity-OE preparation (EB = MHD_PREP_BS / (N+1)^2 elements a block).
// Measured on the 1024^2, N = 4 workload: 128 threads (5 elements, 98 % of the lanes busy) take
// 2.67 ms against 3.16 ms for one-wave blocks (2 elements, 78 %), although the Cholesky barriers
// then span two waves; 256 threads measure the same as 128.
#ifndef MHD_PREP_BS
#define MHD_PREP_BS 128
#endif
template <int P>
struct VP {
  static constexpr int NP = P + 1, NN = NP * NP, EB = MHD_PREP_BS / NN > 0 ? MHD_PREP_BS / NN : 1;
};

// EB elements per block, one thread per node.  The Gram matrix is formed by sum factorisation and packed in
// LDS; a left-looking Cholesky (thread q owns row q, one barrier per column) overwrites it with L,
// and row q of Psi = Phi L^{-T} follows by forward substitution with L read from LDS.  Mode indices
// are compile-time constants in the unrolled loops, and masked arithmetic replaces branches, so
// the steps stay branch-free; the Cholesky dot products run on two accumulators to halve their FMA
// chains (a second accumulator in the substitution as well would cost 50 more VGPRs).
template <int P>
__device__ __forceinline__ void vel_prep_body(const double* __restrict__ rho, double* __restrict__ Psi,
                                                 const HydroTab* __restrict__ H, MeshP mp, long blk) {
  constexpr int NP = P + 1, NN = NP * NP, EB = VP<P>::EB, NL = NN * (NN + 1) / 2;
  constexpr int NPS = NP * (NP + 1) / 2;  // pairs a <= a'
  // LDS (16 KB per 128-thread block at N = 4, so LDS is not what limits the blocks per CU):
  // - sL holds the packed Gram matrix and then L.  Until the Gram rows are written, its first
  //   EB NN entries hold the node weights sw, whose last reads come before the barrier that
  //   precedes the Gram rows.
  // - sH holds the line partials Hm[qj][a][a'] for a <= a', and then the pivot reciprocals srd,
  //   which are first written after the barrier that follows the last reads of the partials.
  // - Masked lanes store to one of eight dummy slots.
  __shared__ double sL[EB][NL], sH[EB][NP][NPS], sV[NP][NP], sdum[8];
  double(*const sw)[NN] = reinterpret_cast<double(*)[NN]>(&sL[0][0]);
  double(*const srd)[NN] = reinterpret_cast<double(*)[NN]>(&sH[0][0][0]);
  const int tid = threadIdx.x, el0 = tid / NN;
  const bool act0 = el0 < EB && blk * EB + el0 < mp.K;
  const int el = act0 ? el0 : 0, q = act0 ? tid - el0 * NN : 0;  // idle lanes shadow lane 0
  const int qi = q % NP, qj = q / NP;
  const long e = blk * EB + el;
  for (int t = tid; t < NP * NP; t += MHD_PREP_BS) sV[t / NP][t % NP] = H->V[t / NP][t % NP];
  if (act0) sw[el][q] = mp.J * H->w[qi] * H->w[qj] * rho[e * NN + q];
  __syncthreads();
  // sum factorisation: Hm[qj][a][a'] = sum_qi W[qj][qi] V[qi][a] V[qi][a'], symmetric in (a, a'),
  // kept for a <= a' (entry p of a line runs over (0, 0..NP-1), (1, 1..NP-1), ...)
  if (act0)
    for (int t = q; t < NP * NPS; t += NN) {
      const int jj = t / NPS;
      int p = t - jj * NPS, a = 0;
      while (p >= NP - a) { p -= NP - a; ++a; }
      const int a2 = a + p;
      double s = 0.0;
#pragma unroll
      for (int ii = 0; ii < NP; ++ii) s += sw[el][jj * NP + ii] * sV[ii][a] * sV[ii][a2];
      sH[el][jj][t - jj * NPS] = s;
    }
  __syncthreads();
  // (LDS stores below go through address selects, not branches: a lane that must not write
  // targets its own dummy slot)
  // Gram row q (shell order): G[q][k'] = sum_qj V[qj][b'] (V[qj][b] Hm[qj][a][a']), k' <= q,
  // packed; row q starts at rq = q (q + 1) / 2, so rq + k <= NL - 1 for every q, k < NN
  const int rq = q * (q + 1) / 2;
  {
    const int ka = mode_a(q), kb = mode_b(q);
    int hx[NP];  // position of the pair (min(a_q, a'), max(a_q, a')) in a line of sH
#pragma unroll
    for (int a2 = 0; a2 < NP; ++a2) {
      const int lo = ka < a2 ? ka : a2, hi = ka < a2 ? a2 : ka;
      hx[a2] = lo * NP - lo * (lo - 1) / 2 + (hi - lo);
    }
    double w[NP][NP];
#pragma unroll
    for (int jj = 0; jj < NP; ++jj)
#pragma unroll
      for (int a2 = 0; a2 < NP; ++a2) w[jj][a2] = sV[jj][kb] * sH[el][jj][hx[a2]];
#pragma unroll
    for (int k2 = 0; k2 < NN; ++k2) {
      double s = 0.0;
#pragma unroll
      for (int jj = 0; jj < NP; ++jj) s += H->V[jj][mode_b(k2)] * w[jj][mode_a(k2)];  // uniform: scalar loads
      *((act0 && k2 <= q) ? &sL[el][rq + k2] : &sdum[tid & 7]) = s;
    }
  }
  __syncthreads();
  // Left-looking Cholesky G = L L^T, one column per step, L written in place over the packed Gram
  // matrix.  Thread q keeps its row of L in registers.  At step k the threads q > k form
  // L[q][k] = (G[q][k] - sum_{m<k} L[q][m] L[k][m]) / L[k][k] with row k read from LDS, and the
  // thread of row k + 1, whose row is then complete up to the diagonal, forms its pivot from its
  // running G[q][q] - sum_m L[q][m]^2.  srd[k] = 1 / L[k][k].
  double Lr[NN];
  double piv = sL[el][rq + q];  // G[q][q]
  {
    const double rk = rsqrt_refined(piv);  // used by row 0 only
    *((act0 && q == 0) ? &sL[el][0] : &sdum[tid & 7]) = piv * rk;
    *((act0 && q == 0) ? &srd[el][0] : &sdum[tid & 7]) = rk;
  }
  __syncthreads();
  // Only the rows q > k read row k; the lanes at or above the diagonal stay masked (measured
  // faster than letting them read and discard; their Lr[k] = 0 is never used).
#pragma unroll
  for (int k = 0; k + 1 < NN; ++k) {
    Lr[k] = 0.0;
    if (q > k) {
      double s0 = sL[el][rq + k], s1 = 0.0;  // G[q][k]
#pragma unroll
      for (int m = 0; m < k; ++m) {
        if (m & 1) s1 -= Lr[m] * sL[el][k * (k + 1) / 2 + m];
        else s0 -= Lr[m] * sL[el][k * (k + 1) / 2 + m];
      }
      Lr[k] = (s0 + s1) * srd[el][k];  // L[q][k]
    }
    *((act0 && q > k) ? &sL[el][rq + k] : &sdum[tid & 7]) = Lr[k];
    piv -= Lr[k] * Lr[k];
    const double rk = rsqrt_refined(piv);  // pivot of row k + 1 (used by that row only)
    *((act0 && q == k + 1) ? &sL[el][rq + q] : &sdum[tid & 7]) = piv * rk;
    *((act0 && q == k + 1) ? &srd[el][k + 1] : &sdum[tid & 7]) = rk;
    __syncthreads();
  }
  // row q of Psi = Phi L^{-T}: forward substitution over the modes with the row in registers
  // (L is read from LDS as broadcasts); Phi[q][k] = V[qi][a_k] V[qj][b_k]
  double vi[NP], vj[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) { vi[a] = sV[qi][a]; vj[a] = sV[qj][a]; }
  // Right-looking order: once psi[k] is final, L[j][k] psi[k] is subtracted from every later
  // entry j.  Each entry receives the same subtractions in the same order as in the row-by-row
  // form (so the results are identical), but the 25 entries are independent chains.
  double psi[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) psi[k] = vi[mode_a(k)] * vj[mode_b(k)];
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    psi[k] *= srd[el][k];
#pragma unroll
    for (int j = k + 1; j < NN; ++j) psi[j] -= sL[el][j * (j + 1) / 2 + k] * psi[k];
  }
  // row q of the element's table, stored directly (rows are 16-byte aligned: psi_row is even)
  if (act0) {
    constexpr long PS = psi_stride(NN), RS = psi_row(NN);
    double2* out = reinterpret_cast<double2*>(Psi + e * PS + q * RS);
#pragma unroll
    for (int k2 = 0; k2 < NN / 2; ++k2) out[k2] = double2{psi[2 * k2], psi[2 * k2 + 1]};
    if (NN % 2) Psi[e * PS + q * RS + NN - 1] = psi[NN - 1];
  }
}

template <int P>
__global__ __launch_bounds__(MHD_PREP_BS) void k_vel_prep(const double* __restrict__ rho, double* __restrict__ Psi,
                                                 const HydroTab* __restrict__ H, MeshP mp) {
  vel_prep_body<P>(rho, Psi, H, mp, (long)blockIdx.x);
}

struct vel_prep_args {
  const double* rho;
  double* Psi;
  const HydroTab* H;
  MeshP mp;
};

template <int P>
__global__ __launch_bounds__(MHD_PREP_BS) void k_vel_prep_rt(const vel_prep_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const vel_prep_args& a = A[r];
  vel_prep_body<P>(gl(a.rho), gl(a.Psi), gl(a.H), a.mp, (long)blockIdx.x - boff[r]);
}

template <int P, int M>
struct VS {
  static constexpr int NP = P + 1, NN = NP * NP, EB = 256 / NN;
  static constexpr int A = M + 2, B = M + 1, AB = A * B, BB = B * B;
};

// Velocity-OE sensor (eq. magnetic-oe-sensor, eq. magnetic-oe-rate, eq. magnetic-oe-factor): one
// thread per GLL_p node, EB elements per block; writes the element's damping factors D_l
// (l = 0..p) to Dfac[K][p+1].  Neighbour velocities are staged per direction in LDS with coalesced
// loads.  u is only read here (the projection kernel that updates it runs afterwards).
// (at N = 4, k = 3 the kernel fits 80 VGPRs and 27 KB of LDS without spills: 6 waves per SIMD)
template <int P, int M, bool R2>
__device__ __forceinline__ void vel_sensor_body(const double* __restrict__ rho, const double* __restrict__ u,
                                                    const double* __restrict__ Bx, const double* __restrict__ By,
                                                    const double* __restrict__ Bz, const double* __restrict__ lines,
                                                    const double* __restrict__ glob, double* __restrict__ Dfac,
                                                    const HydroTab* __restrict__ H, const MagTab* __restrict__ T,
                                                    MeshP mp, double tau, double sM, long blk) {
  using C = VS<P, M>;
  constexpr int NP = C::NP, NN = C::NN, EB = C::EB, A = C::A, B = C::B, AB = C::AB;
  // sbb holds an element's B coefficients (B_x, B_y, B_z at offsets 0, AB, 2 AB) and, once they
  // have been interpolated, its node wave speeds |u_x| + c_A and |u_y| + c_A (offsets 0 and NN);
  // sharing the buffer keeps the block at about 27 KB of LDS at N = 4 (6 blocks per CU)
  constexpr int NSB = 2 * AB + C::BB > 2 * NN ? 2 * AB + C::BB : 2 * NN;
  __shared__ double su[EB][3][NN], sx[EB][6][NN], ssig[EB][2][NP], samp[EB][2][3], ssg[EB][3][NP];
  __shared__ double srow[EB][2][NP];
  __shared__ int scst[EB][3];
  __shared__ double sbb[EB][NSB];
  __shared__ double tD0[NP][NP], tDp[NP][NP], tWP[NP][A], tGP[NP][B], tVP[NP][B], tw[NP], tfr[NP];
  constexpr int NU = R2 ? 2 : 3;  // velocity components (u_z = 0 in the 2D2V system)
  const int tid = threadIdx.x, el = tid / NN, q = tid - el * NN;
  const int qi = q % NP, qj = q / NP;
  const long e = blk * EB + el;
  const bool act = el < EB && e < mp.K;
  int ex, ey;
  elem_xy32(mp, act ? (int)e : 0, ex, ey);
  const long KN = mp.K * NN;
  // node arrays through buffer resources and 32-bit byte offsets (arrays below 2^29 nodes)
  auto uoff = [&](int el_) { return ((unsigned)el_ * NN + q) * 8u; };
  const __amdgpu_buffer_rsrc_t ur[3] = {node_rsrc(u, KN), node_rsrc(u + KN, KN), node_rsrc(u + 2 * KN, KN)};
  for (int t = tid; t < NP * NP; t += 256) {
    tD0[t / NP][t % NP] = H->Dr0[t / NP][t % NP];
    tDp[t / NP][t % NP] = H->Drp[t / NP][t % NP];
  }
  for (int t = tid; t < NP * A; t += 256) tWP[t / A][t % A] = T->I_W_P[t / A][t % A];
  for (int t = tid; t < NP * B; t += 256) {
    tGP[t / B][t % B] = T->I_G_P[t / B][t % B];
    tVP[t / B][t % B] = T->I_V_P[t / B][t % B];
  }
  if (tid < NP) { tw[tid] = H->w[tid]; tfr[tid] = H->fr[tid]; }
  double uu[3] = {0.0, 0.0, 0.0}, rq = 1.0;
  if (act) {
#pragma unroll
    for (int d = 0; d < NU; ++d) { uu[d] = bld(ur[d], uoff((int)e)); su[el][d][q] = uu[d]; }
    rq = bld(node_rsrc(rho, KN), uoff((int)e));
    for (int k = q; k < AB; k += NN) {
      sbb[el][k] = Bx[gix(mp, B, ex, ey, k % A, k / A)];
      sbb[el][AB + k] = By[gix(mp, B, ex, ey, k % B, k / B)];
    }
    for (int k = q; !R2 && k < C::BB; k += NN) sbb[el][2 * AB + k] = Bz[gix(mp, B, ex, ey, k % B, k / B)];
  }
  __syncthreads();
  // shared amplitudes: each component's global and cross-line spreads formed once per element
  for (int c = q; act && c < NU; c += NN) {
    const double gs = glob[c * 3], gmn = glob[c * 3 + 1], gmx = glob[c * 3 + 2];
    const double gm = gs * mp.r4K;
    const double dOm = fmax(gmx - gm, gm - gmn);
    // constant to roundoff: the nodal values agree to 2^10 ulps of the field's size (exact test)
    scst[el][c] = gmx - gmn <= 1024.0 * EPSM * fmax(fabs(gmx), fabs(gmn)) ? 1 : 0;
    const double* rl = lines + (ey * NU + c) * 3;
    const double* cl = lines + ((mp.ny + ex) * NU + c) * 3;
    const double rm = rl[0] * mp.r4nx, cm = cl[0] * mp.r4ny;
    samp[el][0][c] = fmax(fmax(rl[2] - rm, rm - rl[1]), 1e-6 * dOm);
    samp[el][1][c] = fmax(fmax(cl[2] - cm, cm - cl[1]), 1e-6 * dOm);
  }
  double wsx = 0.0, wsy = 0.0;  // node wave speeds
  if (act) {
    double bxv = 0.0, byv = 0.0, bzv = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) s += tWP[qi][i] * sbb[el][j * A + i];
      bxv += tGP[qj][j] * s;
    }
#pragma unroll
    for (int j = 0; j < A; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tGP[qi][i] * sbb[el][AB + j * B + i];
      byv += tWP[qj][j] * s;
    }
#pragma unroll
    for (int j = 0; !R2 && j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tVP[qi][i] * sbb[el][2 * AB + j * B + i];
      bzv += tVP[qj][j] * s;
    }
    const double va = sqrt(bxv * bxv + byv * byv + bzv * bzv) * rsqrt_refined(rq);  // rho > 0
    wsx = fabs(uu[0]) + va;
    wsy = fabs(uu[1]) + va;
  }
  __syncthreads();  // every lane has read the B coefficients
  if (act) { sbb[el][q] = wsx; sbb[el][NN + q] = wsy; }
  // the y neighbours' velocities are loaded into registers here, so that their latency overlaps
  // the x-direction phases (they go to LDS once those are done)
  double uy_nb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (act) {
    const unsigned om = uoff(wrap32(ey - 1, mp.ny) * mp.nx + ex), op = uoff(wrap32(ey + 1, mp.ny) * mp.nx + ex);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      uy_nb[c] = bld(ur[c], om);
      uy_nb[3 + c] = bld(ur[c], op);
    }
  }
#pragma unroll
  for (int D = 0; D < 2; ++D) {
    // neighbours across the faces normal to D: sx rows 0..2 minus side, 3..5 plus side
    if (act) {
      if (D == 0) {
        const unsigned om = uoff(ey * mp.nx + wrap32(ex - 1, mp.nx)), op = uoff(ey * mp.nx + wrap32(ex + 1, mp.nx));
#pragma unroll
        for (int c = 0; c < NU; ++c) {
          sx[el][c][q] = bld(ur[c], om);
          sx[el][3 + c][q] = bld(ur[c], op);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NU; ++c) { sx[el][c][q] = uy_nb[c]; sx[el][3 + c][q] = uy_nb[3 + c]; }
      }
    }
    __syncthreads();
    const int r = D == 0 ? qi : qj, line = D == 0 ? qj : qi;
    double jmp[6];
    if (act) {
      const double wl = 0.5 * tw[line];
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        double a = 0.0, d = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int nk = D == 0 ? line * NP + k : k * NP + line;
          const double own = su[el][c][nk];
          a += tD0[r][k] * own;
          d += tDp[r][k] * own;
          b += tDp[r][k] * sx[el][c][nk];
          cc += tD0[r][k] * sx[el][3 + c][nk];
        }
        const double jm = a - b, jp = cc - d;
        jmp[2 * c] = wl * jm * jm;
        jmp[2 * c + 1] = wl * jp * jp;
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 2 * NU; ++c) sx[el][c][q] = jmp[c];
    }
    __syncthreads();
    // sigma^u: the (r, component) terms spread over the element's threads, then max over components
    {
      double Dsh = 0.0;
#pragma unroll
      for (int c = 0; c < NU; ++c) Dsh = act ? fmax(Dsh, samp[el][D][c]) : 0.0;
      for (int tk = q; act && tk < NU * NP; tk += NN) {
        const int rr = tk % NP, c = tk / NP;
        double v = 0.0;
        if (Dsh > 0.0 && !scst[el][c]) {
          double sm = 0.0, spp = 0.0;
          for (int l = 0; l < NP; ++l) {
            const int nk = D == 0 ? l * NP + rr : rr * NP + l;
            sm += sx[el][2 * c][nk];
            spp += sx[el][2 * c + 1][nk];
          }
          v = tfr[rr] * (sqrt(sm) + sqrt(spp)) / Dsh;
        }
        ssg[el][c][rr] = v;
      }
      if (D == 0)  // row maxima of the node wave speeds, combined over the rows at the end
        for (int t = q; act && t < NP; t += NN) {
          double ax = 0.0, ay = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) { ax = fmax(ax, sbb[el][t * NP + k]); ay = fmax(ay, sbb[el][NN + t * NP + k]); }
          srow[el][0][t] = ax;
          srow[el][1][t] = ay;
        }
    }
    __syncthreads();
    if (act && q < NP) {
      double sig = 0.0;
#pragma unroll
      for (int c = 0; c < NU; ++c) sig = fmax(sig, ssg[el][c][q]);
      ssig[el][D][q] = sig;
    }
    __syncthreads();
  }
  if (act && q <= P) {
    double Dl = 1.0;
    if (q > 0) {
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int l = 0; l < NP; ++l) { ax = fmax(ax, srow[el][0][l]); ay = fmax(ay, srow[el][1][l]); }
      const double lx = (2.0 * P + 1.0) * mp.rhx * ax, ly = (2.0 * P + 1.0) * mp.rhy * ay;
      double sx_ = 0.0, sy_ = 0.0;
      for (int r = 0; r <= q; ++r) { sx_ += ssig[el][0][r]; sy_ += ssig[el][1][r]; }
      Dl = exp(-sM * tau * (lx * sx_ + ly * sy_));
    }
    Dfac[e * NP + q] = Dl;
  }
}

template <int P, int M, bool R2>
__global__ __launch_bounds__(256, (P == 4 && M == 3) ? 6 : 1) void k_vel_sensor(const double* __restrict__ rho, const double* __restrict__ u,
                                                    const double* __restrict__ Bx, const double* __restrict__ By,
                                                    const double* __restrict__ Bz, const double* __restrict__ lines,
                                                    const double* __restrict__ glob, double* __restrict__ Dfac,
                                                    const HydroTab* __restrict__ H, const MagTab* __restrict__ T,
                                                    MeshP mp, double tau, double sM) {
  vel_sensor_body<P, M, R2>(rho, u, Bx, By, Bz, lines, glob, Dfac, H, T, mp, tau, sM, xcd_block());
}

struct vel_sensor_args {
  const double* rho;
  const double* u;
  const double* Bx;
  const double* By;
  const double* Bz;
  const double* lines;
  const double* glob;
  double* Dfac;
  const HydroTab* H;
  const MagTab* T;
  MeshP mp;
  double tau;
  double sM;
};

template <int P, int M, bool R2>
__global__ __launch_bounds__(256, (P == 4 && M == 3) ? 6 : 1) void k_vel_sensor_rt(const vel_sensor_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const vel_sensor_args& a = A[r];
  vel_sensor_body<P, M, R2>(gl(a.rho), gl(a.u), gl(a.Bx), gl(a.By), gl(a.Bz), gl(a.lines), gl(a.glob), gl(a.Dfac), gl(a.H), gl(a.T), a.mp, a.tau, a.sM, (long)blockIdx.x - boff[r]);
}

// Velocity-OE map (eq. magnetic-oe-map) with the prepared basis: one thread per node, EB elements
// per block.  The block's basis tables are copied to LDS first (all of a thread's
// 16-byte loads are issued before the first store; rows keep an odd LDS stride), so the basis is
// read from HBM once; then the coefficients c_k = (u_d, psi_k)_rho (thread = mode) and the shell
// increments at the nodes (thread = node) are formed, and u and e are updated in place.
template <int P, int BS>
struct VPJ {
  static constexpr int NP = P + 1, NN = NP * NP, EB = BS / NN, NNP = NN | 1;
  static constexpr long PS = psi_stride(NN), RS = psi_row(NN);
};

template <int P, int BS, bool R2>
__device__ __forceinline__ void vel_proj_body(const double* __restrict__ rho, double* __restrict__ u,
                                                  double* __restrict__ en, const double* __restrict__ Psi,
                                                  const double* __restrict__ Dfac, const HydroTab* __restrict__ H,
                                                  MeshP mp, double* __restrict__ Uc, long blk) {
  using C = VPJ<P, BS>;
  constexpr int NP = C::NP, NN = C::NN, EB = C::EB, NNP = C::NNP;
  constexpr long PS = C::PS, RS = C::RS;
  __shared__ double sP[EB * NN * NNP];
  __shared__ double sv[EB][3][NN], sc[EB][3][NN], sD[EB][NP];
  const int tid = threadIdx.x, el = tid / NN, q = tid - el * NN;
  const int qi = q % NP, qj = q / NP;
  const long e0 = blk * EB, e = e0 + el;
  const bool act = el < EB && e < mp.K;
  const long KN = mp.K * NN;
  {
    constexpr int NL = (int)((EB * PS / 2 + BS - 1) / BS);
    const long nel = mp.K - e0 < EB ? mp.K - e0 : EB;
    const long n2 = nel * PS / 2;
    const double2* src = reinterpret_cast<const double2*>(Psi + e0 * PS);
    double2 v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const long t = tid + (long)BS * k;
      v[k] = t < n2 ? src[t] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const long t = tid + (long)BS * k;
      if (t < n2) {
        // RS even: both values lie in one row (ee, r), columns c0 and c0 + 1 (padding skipped)
        const int ee = (int)((2 * t) / PS), rem = (int)(2 * t - ee * PS), r = rem / (int)RS, c0 = rem % (int)RS;
        double* d = sP + ee * NN * NNP + r * NNP;
        if (c0 < NN) d[c0] = v[k].x;
        if (c0 + 1 < NN) d[c0 + 1] = v[k].y;
      }
    }
  }
  double rq = 0.0;
  if (act) {
    rq = rho[e * NN + q];
    const double wq = mp.J * H->w[qi] * H->w[qj] * rq;
#pragma unroll
    for (int d = 0; d < (R2 ? 2 : 3); ++d) sv[el][d][q] = wq * u[d * KN + e * NN + q];  // u_z = 0 in 2D2V
    if (q < NP) sD[el][q] = Dfac[e * NP + q];
  }
  __syncthreads();
  const double* Pe = sP + (act ? el : 0) * NN * NNP;  // Pe[n * NNP + k] = psi_k(x_n)
  if (act) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      const double pn = Pe[n * NNP + q];
      s0 += sv[el][0][n] * pn;
      s1 += sv[el][1][n] * pn;
      if (!R2) s2 += sv[el][2][n] * pn;
    }
    sc[el][0][q] = s0; sc[el][1][q] = s1; sc[el][2][q] = s2;
  }
  __syncthreads();
  if (!act) return;
  double wl[3][NP];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int l = 0; l < NP; ++l) wl[d][l] = 0.0;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    const double pk = Pe[q * NNP + k];
    wl[0][shell_of(k)] += sc[el][0][k] * pk;
    wl[1][shell_of(k)] += sc[el][1][k] * pk;
    if (!R2) wl[2][shell_of(k)] += sc[el][2][k] * pk;
  }
  double heat = 0.0, un[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < (R2 ? 2 : 3); ++d) {
    double v = wl[d][0];
#pragma unroll
    for (int l = 1; l < NP; ++l) {
      const double Dl = sD[el][l];
      v += Dl * wl[d][l];
      heat += 0.5 * (1.0 - Dl * Dl) * wl[d][l] * wl[d][l];
    }
    un[d] = v;
  }
  const long n = e * NN + q;
  if (!Uc) {
#pragma unroll
    for (int d = 0; d < (R2 ? 2 : 3); ++d) u[d * KN + n] = un[d];
    en[n] += heat;
  } else {
    // last stage of a Strang step's magnetic substep: the exchange back to the conserved state
    // (section "Local variable exchange") is formed here instead of by a separate pass; the density
    // row of Uc already holds rho, and the primitive copies are not needed afterwards
    const double ev = en[n] + heat;
    Uc[KN + n] = rq * un[0]; Uc[2 * KN + n] = rq * un[1]; Uc[3 * KN + n] = rq * un[2];
    Uc[4 * KN + n] = rq * ev + 0.5 * rq * (un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  }
}

template <int P, int BS, bool R2>
__global__ __launch_bounds__(BS) void k_vel_proj(const double* __restrict__ rho, double* __restrict__ u,
                                                  double* __restrict__ en, const double* __restrict__ Psi,
                                                  const double* __restrict__ Dfac, const HydroTab* __restrict__ H,
                                                  MeshP mp, double* __restrict__ Uc) {
  vel_proj_body<P, BS, R2>(rho, u, en, Psi, Dfac, H, mp, Uc, (long)blockIdx.x);
}

struct vel_proj_args {
  const double* rho;
  double* u;
  double* en;
  const double* Psi;
  const double* Dfac;
  const HydroTab* H;
  MeshP mp;
  double* Uc;
};

template <int P, int BS, bool R2>
__global__ __launch_bounds__(BS) void k_vel_proj_rt(const vel_proj_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const vel_proj_args& a = A[r];
  vel_proj_body<P, BS, R2>(gl(a.rho), gl(a.u), gl(a.en), gl(a.Psi), gl(a.Dfac), gl(a.H), a.mp, gl(a.Uc), (long)blockIdx.x - boff[r]);
}

// ---------------------------------------------------------------------------------------------
// Artificial resistivity (eq. magnetic-ar-sensor, eq. magnetic-ar-coefficient) in two passes.
// Pass 1 (one thread per GLL_p node, B coefficients staged in LDS): each element's tangential
// traces on its four faces at the (m+2) face Gauss points and the element maxima of |u_I| + |B|/sqrt(rho)
// over its GLL_p nodes -> tr[K][8A + 2], trace index ((dir*2 + it)*2 + side)*A + k; dir 0 holds the
// x-faces (it 0: B_y, it 1: B_z), dir 1 the y-faces (it 0: B_x, it 1: B_z); side 0 is the face at -1.
// Pass 2 (one thread per element): squared jumps against the neighbours' traces, sigma^B, R, eta.
// ---------------------------------------------------------------------------------------------
template <int P, int M>
__device__ __forceinline__ void ar_traces_body(const double* __restrict__ rho, const double* __restrict__ u,
                                                   const double* __restrict__ Bx, const double* __restrict__ By,
                                                   const double* __restrict__ Bz, double* __restrict__ tr,
                                                   const MagTab* __restrict__ T, MeshP mp, long blk) {
  constexpr int NP = P + 1, NN = NP * NP, EB = 256 / NN, A = M + 2, B = M + 1, AB = A * B, BB = B * B;
  constexpr int NT = 8 * A + 2;
  __shared__ double sbx[EB][AB], sby[EB][AB], sbz[EB][BB], sv[EB][2][NN];
  __shared__ double tWP[NP][A], tGP[NP][B], tVP[NP][B], tWQ[A][A], tVQ[A][B], tGE[2][B], tVE[2][B];
  const int tid = threadIdx.x, el = tid / NN, q = tid - el * NN, qi = q % NP, qj = q / NP;
  const long e = blk * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  for (int t = tid; t < NP * A; t += 256) tWP[t / A][t % A] = T->I_W_P[t / A][t % A];
  for (int t = tid; t < NP * B; t += 256) {
    tGP[t / B][t % B] = T->I_G_P[t / B][t % B];
    tVP[t / B][t % B] = T->I_V_P[t / B][t % B];
  }
  for (int t = tid; t < A * A; t += 256) tWQ[t / A][t % A] = T->I_W_Q[t / A][t % A];
  for (int t = tid; t < A * B; t += 256) tVQ[t / B][t % B] = T->I_V_Q[t / B][t % B];
  for (int t = tid; t < 2 * B; t += 256) {
    tGE[t / B][t % B] = T->I_G_E[t / B][t % B];
    tVE[t / B][t % B] = T->I_V_E[t / B][t % B];
  }
  if (act) {
    for (int k = q; k < AB; k += NN) {
      sbx[el][k] = Bx[gix(mp, B, ex, ey, k % A, k / A)];  // [j<B][i<A]
      sby[el][k] = By[gix(mp, B, ex, ey, k % B, k / B)];  // [j<A][i<B]
    }
    for (int k = q; k < BB; k += NN) sbz[el][k] = Bz[gix(mp, B, ex, ey, k % B, k / B)];
  }
  __syncthreads();
  double* o = tr + (act ? e : 0) * NT;
  if (act) {
    double bxv = 0.0, byv = 0.0, bzv = 0.0;
    // the outer loops stay rolled: unrolled, the scheduler hoists every LDS operand of the three
    // evaluations at once (170 VGPRs, 2 waves per SIMD)
#pragma unroll 1
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) s += tWP[qi][i] * sbx[el][j * A + i];
      bxv += tGP[qj][j] * s;
    }
#pragma unroll 1
    for (int j = 0; j < A; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tGP[qi][i] * sby[el][j * B + i];
      byv += tWP[qj][j] * s;
    }
#pragma unroll 1
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) s += tVP[qi][i] * sbz[el][j * B + i];
      bzv += tVP[qj][j] * s;
    }
    const double va = sqrt(bxv * bxv + byv * byv + bzv * bzv) * rsqrt_refined(rho[e * NN + q]);  // rho > 0
    sv[el][0][q] = fabs(u[e * NN + q]) + va;
    sv[el][1][q] = fabs(u[KN + e * NN + q]) + va;
    for (int t = q; t < 8 * A; t += NN) {
      const int k = t % A, s = (t / A) % 2, it = (t / (2 * A)) % 2, dir = t / (4 * A);
      double v = 0.0;
      if (it == 1) {  // B_z: GLL_m x GLL_m
        for (int j = 0; j < B; ++j)
          for (int i = 0; i < B; ++i)
            v += (dir == 0 ? tVE[s][i] * tVQ[k][j] : tVQ[k][i] * tVE[s][j]) * sbz[el][j * B + i];
      } else if (dir == 0) {  // B_y on x-faces: Gauss_m in x, GLL_{m+1} in y
        for (int j = 0; j < A; ++j)
          for (int i = 0; i < B; ++i) v += tGE[s][i] * tWQ[k][j] * sby[el][j * B + i];
      } else {  // B_x on y-faces: GLL_{m+1} in x, Gauss_m in y
        for (int j = 0; j < B; ++j)
          for (int i = 0; i < A; ++i) v += tWQ[k][i] * tGE[s][j] * sbx[el][j * A + i];
      }
      o[t] = v;
    }
  }
  __syncthreads();
  if (act && q < 2) {
    double m = 0.0;
    for (int k = 0; k < NN; ++k) m = fmax(m, sv[el][q][k]);
    o[8 * A + q] = m;
  }
}

template <int P, int M>
__global__ __launch_bounds__(256) void k_ar_traces(const double* __restrict__ rho, const double* __restrict__ u,
                                                   const double* __restrict__ Bx, const double* __restrict__ By,
                                                   const double* __restrict__ Bz, double* __restrict__ tr,
                                                   const MagTab* __restrict__ T, MeshP mp) {
  ar_traces_body<P, M>(rho, u, Bx, By, Bz, tr, T, mp, (long)blockIdx.x);
}

struct ar_traces_args {
  const double* rho;
  const double* u;
  const double* Bx;
  const double* By;
  const double* Bz;
  double* tr;
  const MagTab* T;
  MeshP mp;
};

template <int P, int M>
__global__ __launch_bounds__(256) void k_ar_traces_rt(const ar_traces_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const ar_traces_args& a = A[r];
  ar_traces_body<P, M>(gl(a.rho), gl(a.u), gl(a.Bx), gl(a.By), gl(a.Bz), gl(a.tr), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

// bglob[3][3]: (integral, min, max) of B_x, B_y, B_z over the domain.
template <int P, int M>
__device__ __forceinline__ void ar_eta_body(const double* __restrict__ tr, const double* __restrict__ bglob,
                                                double* __restrict__ eta, const MagTab* __restrict__ T, MeshP mp,
                                                double Cs, double Ceta, long blk) {
  constexpr int A = M + 2, NT = 8 * A + 2;
  const long e = blk * blockDim.x + threadIdx.x;
  if (e >= mp.K) return;
  long ex, ey;
  elem_xy(mp, e, ex, ey);
  double dOm[3];
  bool cf[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double mean = bglob[c * 3] / mp.area, mn = bglob[c * 3 + 1], mx = bglob[c * 3 + 2];
    dOm[c] = fmax(mx - mean, mean - mn);
    cf[c] = mx - mn <= 1024.0 * EPSM * fmax(fabs(mx), fabs(mn));  // roundoff-level variation (exact test)
  }
  const double* me = tr + e * NT;
  double R[2];
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    const int t0 = dir == 0 ? 1 : 0;
    const double DB = fmax(cf[t0] ? 0.0 : dOm[t0], cf[2] ? 0.0 : dOm[2]);
    double sig = 0.0;
    if (DB > 0.0) {
      const long em = dir == 0 ? ey * mp.nx + wrapl(ex - 1, mp.nx) : wrapl(ey - 1, mp.ny) * mp.nx + ex;
      const long ep = dir == 0 ? ey * mp.nx + wrapl(ex + 1, mp.nx) : wrapl(ey + 1, mp.ny) * mp.nx + ex;
      const double* tm = tr + em * NT;
      const double* tp = tr + ep * NT;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        if (cf[it == 0 ? t0 : 2]) continue;
        const int b0 = (dir * 2 + it) * 2 * A, b1 = b0 + A;  // side 0 / side 1 blocks
        double sm = 0.0, sp = 0.0;
        for (int k = 0; k < A; ++k) {
          const double jm = me[b0 + k] - tm[b1 + k];
          const double jp = tp[b0 + k] - me[b1 + k];
          sm += 0.5 * T->wq[k] * jm * jm;
          sp += 0.5 * T->wq[k] * jp * jp;
        }
        sig = fmax(sig, (sqrt(sm) + sqrt(sp)) / (2.0 * DB));
      }
    }
    R[dir] = fmin(Cs * sig, 1.0);
  }
  const double v0 = mp.hx / (2.0 * P + 1.0) * me[8 * A] * R[0];
  const double v1 = mp.hy / (2.0 * P + 1.0) * me[8 * A + 1] * R[1];
  eta[e] = Ceta * fmax(v0, v1);
}

template <int P, int M>
__global__ __launch_bounds__(256) void k_ar_eta(const double* __restrict__ tr, const double* __restrict__ bglob,
                                                double* __restrict__ eta, const MagTab* __restrict__ T, MeshP mp,
                                                double Cs, double Ceta) {
  ar_eta_body<P, M>(tr, bglob, eta, T, mp, Cs, Ceta, (long)blockIdx.x);
}

struct ar_eta_args {
  const double* tr;
  const double* bglob;
  double* eta;
  const MagTab* T;
  MeshP mp;
  double Cs;
  double Ceta;
};

template <int P, int M>
__global__ __launch_bounds__(256) void k_ar_eta_rt(const ar_eta_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const ar_eta_args& a = A[r];
  ar_eta_body<P, M>(gl(a.tr), gl(a.bglob), gl(a.eta), gl(a.T), a.mp, a.Cs, a.Ceta, (long)blockIdx.x - boff[r]);
}

// per-element exact integral and owned-node min / max of each B component -> [K][3][3]
template <int M>
__device__ __forceinline__ void B_stats_body(const double* __restrict__ Bx, const double* __restrict__ By,
                                                 const double* __restrict__ Bz, double* __restrict__ stats,
                                                 const MagTab* __restrict__ T, MeshP mp, long blk) {
  constexpr int A = M + 2, B = M + 1;
  const long e = blk * blockDim.x + threadIdx.x;
  if (e >= mp.K) return;
  long ex, ey;
  elem_xy(mp, e, ex, ey);
  double s[3] = {0, 0, 0}, mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  // extrema over the element's own DOFs (its upper shared nodes belong to the next element); on a
  // mirror-walled mesh the box's last column / row of elements also takes the box's wall DOFs
  const bool wx = (mp.walls & 1) && ex == mp.bx - 1, wy = (mp.walls & 2) && ey == mp.by - 1;
  // outer loops rolled: fully unrolled, the three loops keep every load in flight at once (about
  // 190 VGPRs, 2 waves per SIMD instead of 6)
#pragma unroll 1
  for (int j = 0; j < B; ++j)
    for (int i = 0; i < A; ++i) {
      const double v = Bx[gix(mp, B, ex, ey, i, j)];
      s[0] += T->ww[i] * T->wg[j] * v;
      if (i < B || wx) { mn[0] = fmin(mn[0], v); mx[0] = fmax(mx[0], v); }
    }
#pragma unroll 1
  for (int j = 0; j < A; ++j)
    for (int i = 0; i < B; ++i) {
      const double v = By[gix(mp, B, ex, ey, i, j)];
      s[1] += T->wg[i] * T->ww[j] * v;
      if (j < B || wy) { mn[1] = fmin(mn[1], v); mx[1] = fmax(mx[1], v); }
    }
#pragma unroll 1
  for (int j = 0; j < B; ++j)
    for (int i = 0; i < B; ++i) {
      const double v = Bz[gix(mp, B, ex, ey, i, j)];
      s[2] += T->wv[i] * T->wv[j] * v;
      mn[2] = fmin(mn[2], v); mx[2] = fmax(mx[2], v);
    }
  for (int c = 0; c < 3; ++c) {
    stats[(e * 3 + c) * 3] = mp.J * s[c];
    stats[(e * 3 + c) * 3 + 1] = mn[c];
    stats[(e * 3 + c) * 3 + 2] = mx[c];
  }
}

template <int M>
__global__ __launch_bounds__(256) void k_B_stats(const double* __restrict__ Bx, const double* __restrict__ By,
                                                 const double* __restrict__ Bz, double* __restrict__ stats,
                                                 const MagTab* __restrict__ T, MeshP mp) {
  B_stats_body<M>(Bx, By, Bz, stats, T, mp, (long)blockIdx.x);
}

struct B_stats_args {
  const double* Bx;
  const double* By;
  const double* Bz;
  double* stats;
  const MagTab* T;
  MeshP mp;
};

template <int M>
__global__ __launch_bounds__(256) void k_B_stats_rt(const B_stats_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const B_stats_args& a = A[r];
  B_stats_body<M>(gl(a.Bx), gl(a.By), gl(a.Bz), gl(a.stats), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

}  // namespace

// gather of per-element loads at shared nodes and division by the lumped weights
template <int M, bool R2>
__device__ __forceinline__ void gather_body(const double* __restrict__ Lx, const double* __restrict__ Ly,
                                                const double* __restrict__ Lz, double* __restrict__ Ox,
                                                double* __restrict__ Oy, double* __restrict__ Oz,
                                                const MagTab* __restrict__ T, MeshP mp, long blk) {
  constexpr int A = M + 2, B = M + 1, AA = A * A, AB = A * B;
  const int NX = mp.nx * B;
  const long G = (long)NX * mp.ny * B;  // below 2^29 (mhd25_init)
  const long g = blk * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int gy = (int)row_of(mp, g / B), gx = (int)g - gy * NX;  // g / (nx B) = (g / B) / nx
  const int ex = gx / B, ey = gy / B;
  const int i = gx - ex * B, j = gy - ey * B;
  const long e = (long)ey * mp.nx + ex;
  const long eL = (long)ey * mp.nx + wrap32(ex - 1, mp.nx), eD = (long)wrap32(ey - 1, mp.ny) * mp.nx + ex;
  const long eLD = (long)wrap32(ey - 1, mp.ny) * mp.nx + wrap32(ex - 1, mp.nx);
  {  // W node
    double s = Lz[e * AA + j * A + i];
    if (i == 0) s += Lz[eL * AA + j * A + (A - 1)];
    if (j == 0) s += Lz[eD * AA + (A - 1) * A + i];
    if (i == 0 && j == 0) s += Lz[eLD * AA + (A - 1) * A + (A - 1)];
    Oz[g] = s * T->rjw[0][j][i];
  }
  if (R2) return;  // the 2D2V system has no in-plane J or E
  {  // N_x node: Gauss in x (i), GLL in y (j); local index j*B + i
    double s = Lx[e * AB + j * B + i];
    if (j == 0) s += Lx[eD * AB + (A - 1) * B + i];
    Ox[g] = s * T->rjw[1][j][i];
  }
  {  // N_y node: GLL in x (i), Gauss in y (j); local index j*A + i
    double s = Ly[e * AB + j * A + i];
    if (i == 0) s += Ly[eL * AB + j * A + (A - 1)];
    Oy[g] = s * T->rjw[2][j][i];
  }
}

template <int M, bool R2>
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ Lx, const double* __restrict__ Ly,
                                                const double* __restrict__ Lz, double* __restrict__ Ox,
                                                double* __restrict__ Oy, double* __restrict__ Oz,
                                                const MagTab* __restrict__ T, MeshP mp) {
  gather_body<M, R2>(Lx, Ly, Lz, Ox, Oy, Oz, T, mp, (long)blockIdx.x);
}

struct gather_args {
  const double* Lx;
  const double* Ly;
  const double* Lz;
  double* Ox;
  double* Oy;
  double* Oz;
  const MagTab* T;
  MeshP mp;
};

template <int M, bool R2>
__global__ __launch_bounds__(256) void k_gather_rt(const gather_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const gather_args& a = A[r];
  gather_body<M, R2>(gl(a.Lx), gl(a.Ly), gl(a.Lz), gl(a.Ox), gl(a.Oy), gl(a.Oz), gl(a.T), a.mp, (long)blockIdx.x - boff[r]);
}

// Local-to-global maps of the six magnetic node sets of each element (B_x, B_y, B_z, W, N_x, N_y;
// local order [j][i], i fastest), formed with the kernels' own grid index gix.  One thread per element.
template <int M>
__global__ __launch_bounds__(256) void k_dof_maps(int32_t* __restrict__ dof, MeshP mp) {
  constexpr int A = M + 2, B = M + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp.K) return;
  long ex, ey;
  elem_xy(mp, e, ex, ey);
  const int ni[6] = {A, B, B, A, B, A}, nj[6] = {B, A, B, A, A, B};
  long off = 0;
  for (int s = 0; s < 6; ++s) {
    const int n = ni[s] * nj[s];
    int32_t* o = dof + off + e * n;
    for (int j = 0; j < nj[s]; ++j)
      for (int i = 0; i < ni[s]; ++i) o[j * ni[s] + i] = (int32_t)gix(mp, B, ex, ey, i, j);
    off += mp.K * n;
  }
}

// Admissibility test of a magnetic-substep input: rho > 0, e > 0 (p = (gamma - 1) rho e > 0) and
// finite u at every node, finite magnetic grids.  A failure sets bit 1 of flag[1].
__global__ __launch_bounds__(256) void k_check_mag(const double* __restrict__ rho, const double* __restrict__ e,
                                                   const double* __restrict__ u, long KN, const double* __restrict__ Bx,
                                                   const double* __restrict__ By, const double* __restrict__ Bz, long G,
                                                   int* __restrict__ flag) {
  const long n = KN > G ? KN : G;
  bool ok = true;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    if (k < KN) {
      const double r = rho[k], en = e[k];
      ok = ok && r > 0.0 && en > 0.0 && r <= DBL_MAX && en <= DBL_MAX && fabs(u[k]) <= DBL_MAX &&
           fabs(u[KN + k]) <= DBL_MAX && fabs(u[2 * KN + k]) <= DBL_MAX;
    }
    if (k < G) ok = ok && fabs(Bx[k]) <= DBL_MAX && fabs(By[k]) <= DBL_MAX && fabs(Bz[k]) <= DBL_MAX;
  }
  if (!ok) atomicOr(flag + 1, 2);
}

__device__ __forceinline__ void to_primitive_node(const double* __restrict__ U, double* __restrict__ rho,
                                                  double* __restrict__ e, double* __restrict__ u, long n, long k) {
  const double r = U[k], ux = U[n + k] / r, uy = U[2 * n + k] / r, uz = U[3 * n + k] / r;
  rho[k] = r; u[k] = ux; u[n + k] = uy; u[2 * n + k] = uz;
  e[k] = (U[4 * n + k] - 0.5 * r * (ux * ux + uy * uy + uz * uz)) / r;
}

__device__ __forceinline__ void to_conservative_node(const double* __restrict__ rho, const double* __restrict__ e,
                                                     const double* __restrict__ u, double* __restrict__ U, long n,
                                                     long k) {
  const double r = rho[k], ux = u[k], uy = u[n + k], uz = u[2 * n + k];
  U[k] = r; U[n + k] = r * ux; U[2 * n + k] = r * uy; U[3 * n + k] = r * uz;
  U[4 * n + k] = r * e[k] + 0.5 * r * (ux * ux + uy * uy + uz * uz);
}

__global__ void k_to_primitive(const double* __restrict__ U, double* __restrict__ rho, double* __restrict__ e,
                               double* __restrict__ u, long n) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    to_primitive_node(U, rho, e, u, n, k);
}

__global__ void k_to_conservative(const double* __restrict__ rho, const double* __restrict__ e,
                                  const double* __restrict__ u, double* __restrict__ U, long n) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    to_conservative_node(rho, e, u, U, n, k);
}

// B_par = (-d_y A, d_x A) for A on the E_z grid
template <int M>
__global__ void k_B_from_potential(const double* __restrict__ Az, double* __restrict__ Bx, double* __restrict__ By,
                                   const MagTab* __restrict__ T, MeshP mp) {
  constexpr int A = M + 2, B = M + 1;
  const long NX = (long)mp.nx * B, G = NX * mp.ny * B;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const long gy = row_of(mp, g / B), gx = g - gy * NX;  // g / (nx B) = (g / B) / nx
  const long ex = gx / B, ey = gy / B;
  const int i = gx - ex * B, j = gy - ey * B;
  double bx = 0.0, by = 0.0;
  for (int k = 0; k < A; ++k) {
    bx += T->D_W_G[j][k] * Az[gix(mp, B, ex, ey, i, k)];  // B_x node: GLL i, Gauss j
    by += T->D_W_G[i][k] * Az[gix(mp, B, ex, ey, k, j)];  // B_y node: Gauss i, GLL j
  }
  Bx[g] = -(2.0 / mp.hy) * bx;
  By[g] = (2.0 / mp.hx) * by;
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
int line_global_reduce(mhd25_ctx* c, const double* stats, int nc, const int* flag);
int dcopy(mhd25_ctx* c, const double* a, double* b, long n);

static int chk(mhd25_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { c->err = std::string(what) + ": " + hipGetErrorString(e); return -2; }
  return 0;
}

hipEvent_t* timing_slot(mhd25_ctx* c, int kid);
// HIP-event timing of one launch (kernel id kid) when the context's timing is on
#define T_BEGIN(kid)                                                   \
  hipEvent_t* ev_ = c->timing ? timing_slot(c, kid) : nullptr;         \
  if (ev_) hipEventRecord(ev_[0], c->stream)
#define T_END() \
  if (ev_) hipEventRecord(ev_[1], c->stream)

#define DISPATCH_PM(p, m, F)                                                                              \
  if (p == 1 && m == 0) { F(1, 0); } else if (p == 1 && m == 1) { F(1, 1); }                              \
  else if (p == 2 && m == 1) { F(2, 1); } else if (p == 2 && m == 2) { F(2, 2); }                         \
  else if (p == 3 && m == 2) { F(3, 2); } else if (p == 3 && m == 3) { F(3, 3); }                         \
  else if (p == 4 && m == 3) { F(4, 3); } else if (p == 4 && m == 4) { F(4, 4); }                         \
  else if (p == 5 && m == 4) { F(5, 4); } else if (p == 5 && m == 5) { F(5, 5); }                         \
  else if (p == 6 && m == 5) { F(6, 5); } else if (p == 6 && m == 6) { F(6, 6); }                         \
  else return -4;

#define DISPATCH_M(m, F) \
  switch (m) { case 0: F(0); break; case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; \
               case 4: F(4); break; case 5: F(5); break; case 6: F(6); break; default: return -4; }

// template keys of run-table records: degree p, magnetic degree m, 2D2V flag, mode
static int mkey(int p, int m, bool r2, int mode = 0) { return p * 1000 + m * 100 + (r2 ? 10 : 0) + mode; }

static long mblocks(int p, int m, long K, int bs = 256) {
  const int nn = (p + 1) * (p + 1), aa = (m + 2) * (m + 2);
  const int eb = bs / (nn > aa ? nn : aa);
  return (K + eb - 1) / eb;
}

// threads per block of the element-load and update kernels (measured on the 1024^2, N = 4, k = 3
// workload: 128-thread blocks make the E loads 6 % faster, being limited by their LDS use at 256;
// the J loads and the update run slightly slower with 128)
#ifndef MHD_JL_BS
#define MHD_JL_BS 256
#endif
#ifndef MHD_EL_BS
#define MHD_EL_BS 128
#endif
#ifndef MHD_MU_BS
#define MHD_MU_BS 256
#endif
// threads per block of the velocity-OE projection (its per-element basis tile in LDS sets how
// many blocks share a CU)
#ifndef MHD_VP_BS
#define MHD_VP_BS 128
#endif

// r2: the 2D2V reduced system (only J_z and E_z are formed; the in-plane grids are not written)
// loads: the per-element load workspace, K (2 (m+2)(m+1) + (m+2)^2) doubles
static int reconstruct_JE_ws(mhd25_ctx* c, const double* u, const double* Bx, const double* By, const double* Bz,
                             const double* eta, double* JE, bool r2, double* loads) {
  const long K = c->mp.K, G = c->G;
  const int a = c->m + 2, b = c->m + 1;
  double* Lx = loads;
  double* Ly = Lx + K * a * b;
  double* Lz = Ly + K * a * b;
  const long nbj = mblocks(c->p, c->m, K, MHD_JL_BS), nbe = mblocks(c->p, c->m, K, MHD_EL_BS);
  const long gb = (G + 255) / 256;
  if (c->rec) {
    const int k = mkey(c->p, c->m, r2);
    rt_record(c, RT_J_LOADS, k, nbj, J_loads_args{Bx, By, Bz, Lx, Ly, Lz, c->d_mt, c->mp});
    rt_record(c, RT_GATHER, k, gb, gather_args{Lx, Ly, Lz, JE, JE + G, JE + 2 * G, c->d_mt, c->mp});
    rt_record(c, RT_E_LOADS, k, nbe,
              E_loads_args{u, Bx, By, Bz, JE, JE + G, JE + 2 * G, eta, Lx, Ly, Lz, c->d_mt, c->mp});
    rt_record(c, RT_GATHER, k, gb, gather_args{Lx, Ly, Lz, JE + 3 * G, JE + 4 * G, JE + 5 * G, c->d_mt, c->mp});
    return 0;
  }
#define LJ(P, M)                                                                                                    \
  if (r2) hipLaunchKernelGGL((k_J_loads<P, M, MHD_JL_BS, true>), dim3(nbj), dim3(MHD_JL_BS), 0, c->stream, Bx, By, \
                             Bz, Lx, Ly, Lz, c->d_mt, c->mp);                                                       \
  else hipLaunchKernelGGL((k_J_loads<P, M, MHD_JL_BS, false>), dim3(nbj), dim3(MHD_JL_BS), 0, c->stream, Bx, By, Bz, \
                          Lx, Ly, Lz, c->d_mt, c->mp)
  {
    T_BEGIN(7);
    DISPATCH_PM(c->p, c->m, LJ);
    T_END();
  }
#undef LJ
#define GJ(M)                                                                                                       \
  if (r2) hipLaunchKernelGGL((k_gather<M, true>), dim3(gb), dim3(256), 0, c->stream, Lx, Ly, Lz, JE, JE + G,       \
                             JE + 2 * G, c->d_mt, c->mp);                                                           \
  else hipLaunchKernelGGL((k_gather<M, false>), dim3(gb), dim3(256), 0, c->stream, Lx, Ly, Lz, JE, JE + G,         \
                          JE + 2 * G, c->d_mt, c->mp)
  {
    T_BEGIN(8);
    DISPATCH_M(c->m, GJ);
    T_END();
  }
#undef GJ
#define LE(P, M)                                                                                                    \
  if (r2) hipLaunchKernelGGL((k_E_loads<P, M, MHD_EL_BS, true>), dim3(nbe), dim3(MHD_EL_BS), 0, c->stream, u, Bx,  \
                             By, Bz, JE, JE + G, JE + 2 * G, eta, Lx, Ly, Lz, c->d_mt, c->mp);                      \
  else hipLaunchKernelGGL((k_E_loads<P, M, MHD_EL_BS, false>), dim3(nbe), dim3(MHD_EL_BS), 0, c->stream, u, Bx, By, \
                          Bz, JE, JE + G, JE + 2 * G, eta, Lx, Ly, Lz, c->d_mt, c->mp)
  {
    T_BEGIN(5);
    DISPATCH_PM(c->p, c->m, LE);
    T_END();
  }
#undef LE
#define GE(M)                                                                                                       \
  if (r2) hipLaunchKernelGGL((k_gather<M, true>), dim3(gb), dim3(256), 0, c->stream, Lx, Ly, Lz, JE + 3 * G,       \
                             JE + 4 * G, JE + 5 * G, c->d_mt, c->mp);                                               \
  else hipLaunchKernelGGL((k_gather<M, false>), dim3(gb), dim3(256), 0, c->stream, Lx, Ly, Lz, JE + 3 * G,         \
                          JE + 4 * G, JE + 5 * G, c->d_mt, c->mp)
  {
    T_BEGIN(8);
    DISPATCH_M(c->m, GE);
    T_END();
  }
#undef GE
  return chk(c, "reconstruct launch");
}

int mag_reconstruct_JE(mhd25_ctx* c, const double* u, const double* Bx, const double* By, const double* Bz,
                       const double* eta, double* JE, bool r2) {
  return reconstruct_JE_ws(c, u, Bx, By, Bz, eta, JE, r2, c->loads);
}

int mag_update(mhd25_ctx* c, const MagIO& io, int mode) {
  const long nb = mblocks(c->p, c->m, c->mp.K, MHD_MU_BS);
  const bool r2 = c->opt.reduced_2d2v != 0;
  if (c->rec) { rt_record(c, RT_MAG_UPDATE, mkey(c->p, c->m, r2, mode), nb, mag_update_args{io, c->d_mt, c->mp}); return 0; }
#define U0(P, M)                                                                                                    \
  if (r2) hipLaunchKernelGGL((k_mag_update<P, M, 0, MHD_MU_BS, true>), dim3(nb), dim3(MHD_MU_BS), 0, c->stream, io, \
                             c->d_mt, c->mp);                                                                        \
  else hipLaunchKernelGGL((k_mag_update<P, M, 0, MHD_MU_BS, false>), dim3(nb), dim3(MHD_MU_BS), 0, c->stream, io,   \
                          c->d_mt, c->mp)
#define U1(P, M)                                                                                                    \
  if (r2) hipLaunchKernelGGL((k_mag_update<P, M, 1, MHD_MU_BS, true>), dim3(nb), dim3(MHD_MU_BS), 0, c->stream, io, \
                             c->d_mt, c->mp);                                                                        \
  else hipLaunchKernelGGL((k_mag_update<P, M, 1, MHD_MU_BS, false>), dim3(nb), dim3(MHD_MU_BS), 0, c->stream, io,   \
                          c->d_mt, c->mp)
  T_BEGIN(2);
  if (mode == 0) {
    DISPATCH_PM(c->p, c->m, U0);
  } else {
    DISPATCH_PM(c->p, c->m, U1);
  }
  T_END();
#undef U0
#undef U1
  return chk(c, "magnetic update launch");
}

static int vp_eb(int p) {
  switch (p) { case 1: return VP<1>::EB; case 2: return VP<2>::EB; case 3: return VP<3>::EB;
               case 4: return VP<4>::EB; case 5: return VP<5>::EB; default: return VP<6>::EB; }
}

int mag_velocity_prep(mhd25_ctx* c, const double* rho) {
  const long K = c->mp.K;
  const long nn = (long)(c->p + 1) * (c->p + 1);
  (void)nn;
  if (!c->psi) { c->err = "velocity-OE basis not allocated"; return -2; }
  if (c->rec) {
    rt_record(c, RT_VEL_PREP, c->p, (K + vp_eb(c->p) - 1) / vp_eb(c->p),
              vel_prep_args{rho, c->psi, c->d_ht, c->mp});
    return 0;
  }
#define VPR(P) hipLaunchKernelGGL((k_vel_prep<P>), dim3((K + VP<P>::EB - 1) / VP<P>::EB), dim3(MHD_PREP_BS), 0, c->stream, rho, \
                                  c->psi, c->d_ht, c->mp)
  T_BEGIN(4);
  switch (c->p) { case 1: VPR(1); break; case 2: VPR(2); break; case 3: VPR(3); break; case 4: VPR(4); break;
                  case 5: VPR(5); break; case 6: VPR(6); break; default: return -4; }
  T_END();
#undef VPR
  return chk(c, "velocity OE prep launch");
}

int mag_velocity_apply(mhd25_ctx* c, double tau, const double* rho, double* u, double* e, const double* Bx,
                       const double* By, const double* Bz, bool stats_ready, double* Uc) {
  const long K = c->mp.K;
  const int nn = (c->p + 1) * (c->p + 1), eb = 256 / nn, eb2 = MHD_VP_BS / nn;
  const long nb = (K + eb - 1) / eb, nb2 = (K + eb2 - 1) / eb2;
  const bool r2 = c->opt.reduced_2d2v != 0;
  const int nu = r2 ? 2 : 3;  // velocity components carried
  if (!stats_ready && !c->rec) {
#define FS(P)                                                                                                       \
  if (r2) hipLaunchKernelGGL((k_field_stats<P, 2>), dim3(nb), dim3(256), 0, c->stream, u, c->stats, c->d_mt, c->mp); \
  else hipLaunchKernelGGL((k_field_stats<P, 3>), dim3(nb), dim3(256), 0, c->stream, u, c->stats, c->d_mt, c->mp)
    switch (c->p) { case 1: FS(1); break; case 2: FS(2); break; case 3: FS(3); break; case 4: FS(4); break;
                    case 5: FS(5); break; case 6: FS(6); break; default: return -4; }
#undef FS
  }
  line_global_reduce(c, c->stats, nu, nullptr);
  if (c->rec) {
    if (!stats_ready) { c->err = "run-table plan: velocity statistics must come from the update"; return -2; }
    rt_record(c, RT_VEL_SENSOR, mkey(c->p, c->m, r2), nb,
              vel_sensor_args{rho, u, Bx, By, Bz, c->lines, c->glob, c->dfac, c->d_ht, c->d_mt, c->mp, tau, c->opt.s_M});
    rt_record(c, RT_VEL_PROJ, mkey(c->p, c->m, r2), nb2, vel_proj_args{rho, u, e, c->psi, c->dfac, c->d_ht, c->mp, Uc});
    return 0;
  }
#define VSN(P, M)                                                                                                   \
  if (r2) hipLaunchKernelGGL((k_vel_sensor<P, M, true>), dim3(nb), dim3(256), 0, c->stream, rho, u, Bx, By, Bz,    \
                             c->lines, c->glob, c->dfac, c->d_ht, c->d_mt, c->mp, tau, c->opt.s_M);                 \
  else hipLaunchKernelGGL((k_vel_sensor<P, M, false>), dim3(nb), dim3(256), 0, c->stream, rho, u, Bx, By, Bz,      \
                          c->lines, c->glob, c->dfac, c->d_ht, c->d_mt, c->mp, tau, c->opt.s_M)
  {
    T_BEGIN(6);
    DISPATCH_PM(c->p, c->m, VSN);
    T_END();
  }
#undef VSN
#define VPR(P)                                                                                                      \
  if (r2) hipLaunchKernelGGL((k_vel_proj<P, MHD_VP_BS, true>), dim3(nb2), dim3(MHD_VP_BS), 0, c->stream, rho, u, e, \
                             c->psi, c->dfac, c->d_ht, c->mp, Uc);                                                    \
  else hipLaunchKernelGGL((k_vel_proj<P, MHD_VP_BS, false>), dim3(nb2), dim3(MHD_VP_BS), 0, c->stream, rho, u, e,   \
                          c->psi, c->dfac, c->d_ht, c->mp, Uc)
  {
    T_BEGIN(3);
    switch (c->p) { case 1: VPR(1); break; case 2: VPR(2); break; case 3: VPR(3); break; case 4: VPR(4); break;
                    case 5: VPR(5); break; case 6: VPR(6); break; default: return -4; }
    T_END();
  }
#undef VPR
  return chk(c, "velocity OE launch");
}

int mag_velocity_oe(mhd25_ctx* c, double tau, const double* rho, double* u, double* e, const double* Bx,
                    const double* By, const double* Bz) {
  int r = mag_velocity_prep(c, rho);
  if (r) return r;
  return mag_velocity_apply(c, tau, rho, u, e, Bx, By, Bz, false, nullptr);
}

int mag_ar_eta(mhd25_ctx* c, const double* rho, const double* u, const double* Bx, const double* By,
               const double* Bz, double* eta) {
  const long K = c->mp.K;
  const long nb = (K + 255) / 256;
  if (c->rec) {
    const long eb = 256 / ((c->p + 1) * (c->p + 1));
    rt_record(c, RT_B_STATS, c->m, nb, B_stats_args{Bx, By, Bz, c->stats, c->d_mt, c->mp});
    line_global_reduce(c, c->stats, 3, nullptr);
    rt_record(c, RT_AR_TRACES, mkey(c->p, c->m, false), (K + eb - 1) / eb,
              ar_traces_args{rho, u, Bx, By, Bz, c->artr, c->d_mt, c->mp});
    rt_record(c, RT_AR_ETA, mkey(c->p, c->m, false), nb,
              ar_eta_args{c->artr, c->glob, eta, c->d_mt, c->mp, c->opt.C_s, c->opt.C_eta});
    return 0;
  }
#define BS(M) hipLaunchKernelGGL((k_B_stats<M>), dim3(nb), dim3(256), 0, c->stream, Bx, By, Bz, c->stats, c->d_mt, c->mp)
  DISPATCH_M(c->m, BS);
#undef BS
  line_global_reduce(c, c->stats, 3, nullptr);
  const long eb = 256 / ((c->p + 1) * (c->p + 1));
  const long nb1 = (K + eb - 1) / eb;
#define ART(P, M) hipLaunchKernelGGL((k_ar_traces<P, M>), dim3(nb1), dim3(256), 0, c->stream, rho, u, Bx, By, Bz, c->artr, \
                                     c->d_mt, c->mp)
  {
    T_BEGIN(9);
    DISPATCH_PM(c->p, c->m, ART);
    T_END();
  }
#undef ART
#define AR(P, M) hipLaunchKernelGGL((k_ar_eta<P, M>), dim3(nb), dim3(256), 0, c->stream, c->artr, c->glob, eta, c->d_mt, \
                                    c->mp, c->opt.C_s, c->opt.C_eta)
  DISPATCH_PM(c->p, c->m, AR);
#undef AR
  return chk(c, "A.R. launch");
}

struct prim_args {
  const double* U;
  double *rho, *e, *u;
  long n;
};

int mag_to_primitive(mhd25_ctx* c, const double* U, double* rho, double* e, double* u) {
  const long n = c->mp.K * c->nn;
  long nb = (n + 255) / 256; if (nb > 65536) nb = 65536;
  if (c->rec) { rt_record(c, RT_TO_PRIM, 0, nb, prim_args{U, rho, e, u, n}); return 0; }
  hipLaunchKernelGGL(k_to_primitive, dim3(nb), dim3(256), 0, c->stream, U, rho, e, u, n);
  return chk(c, "exchange launch");
}

int mag_to_conservative(mhd25_ctx* c, const double* rho, const double* e, const double* u, double* U) {
  const long n = c->mp.K * c->nn;
  long nb = (n + 255) / 256; if (nb > 65536) nb = 65536;
  if (c->rec) { rt_record(c, RT_TO_CONS, 0, nb, prim_args{U, const_cast<double*>(rho), const_cast<double*>(e), const_cast<double*>(u), n}); return 0; }
  hipLaunchKernelGGL(k_to_conservative, dim3(nb), dim3(256), 0, c->stream, rho, e, u, U, n);
  return chk(c, "exchange launch");
}

int entry_clear(mhd25_ctx* c);

int mag_dof_maps(mhd25_ctx* c, int32_t* dof) {
  const long nb = (c->mp.K + 255) / 256;
#define DM(M) hipLaunchKernelGGL((k_dof_maps<M>), dim3(nb), dim3(256), 0, c->stream, dof, c->mp)
  DISPATCH_M(c->m, DM);
#undef DM
  return chk(c, "dof map launch");
}

// clears the entry word flag[1], then tests the magnetic-substep input into it
int mag_check_input(mhd25_ctx* c, const double* rho, const double* e, const double* u, const double* Bx,
                    const double* By, const double* Bz) {
  const long KN = c->mp.K * c->nn, n = KN > c->G ? KN : c->G;
  long nb = (n + 255) / 256; if (nb > 65536) nb = 65536;
  if (const int r = entry_clear(c)) return r;
  hipLaunchKernelGGL(k_check_mag, dim3(nb), dim3(256), 0, c->stream, rho, e, u, KN, Bx, By, Bz, c->G, c->d_flag);
  return chk(c, "input check launch");
}

int mag_B_from_potential(mhd25_ctx* c, const double* A, double* Bx, double* By) {
  const long gb = (c->G + 255) / 256;
#define BP(M) hipLaunchKernelGGL((k_B_from_potential<M>), dim3(gb), dim3(256), 0, c->stream, A, Bx, By, c->d_mt, c->mp)
  DISPATCH_M(c->m, BP);
#undef BP
  return chk(c, "potential launch");
}

// ---------------------------------------------------------------------------------------------
// Run-table launches of this file's kernels (batched ensembles).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_to_primitive_rt(const prim_args* __restrict__ A, const int* __restrict__ boff,
                                                         int nr) {
  const int r = rt_run(boff, nr);
  const prim_args& a = A[r];
  const long stride = (long)(boff[r + 1] - boff[r]) * blockDim.x;
  for (long k = (long)(blockIdx.x - boff[r]) * blockDim.x + threadIdx.x; k < a.n; k += stride)
    to_primitive_node(gl(a.U), gl(a.rho), gl(a.e), gl(a.u), a.n, k);
}

__global__ __launch_bounds__(256) void k_to_conservative_rt(const prim_args* __restrict__ A,
                                                            const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const prim_args& a = A[r];
  const long stride = (long)(boff[r + 1] - boff[r]) * blockDim.x;
  for (long k = (long)(blockIdx.x - boff[r]) * blockDim.x + threadIdx.x; k < a.n; k += stride)
    to_conservative_node(gl(a.rho), gl(a.e), gl(a.u), const_cast<double*>(gl(a.U)), a.n, k);
}

int magnetic_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s) {
  const dim3 g((unsigned)nblocks);
  const int p = h.key / 1000, m = (h.key / 100) % 10, mode = h.key % 10;
  const bool r2 = (h.key / 10) % 10 != 0;
  switch (h.kind) {
    case RT_J_LOADS: {
      const J_loads_args* A = (const J_loads_args*)dargs;
#define F(P, M)                                                                                                     \
  if (r2) hipLaunchKernelGGL((k_J_loads_rt<P, M, MHD_JL_BS, true>), g, dim3(MHD_JL_BS), 0, s, A, dboff, nr);       \
  else hipLaunchKernelGGL((k_J_loads_rt<P, M, MHD_JL_BS, false>), g, dim3(MHD_JL_BS), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_E_LOADS: {
      const E_loads_args* A = (const E_loads_args*)dargs;
#define F(P, M)                                                                                                     \
  if (r2) hipLaunchKernelGGL((k_E_loads_rt<P, M, MHD_EL_BS, true>), g, dim3(MHD_EL_BS), 0, s, A, dboff, nr);       \
  else hipLaunchKernelGGL((k_E_loads_rt<P, M, MHD_EL_BS, false>), g, dim3(MHD_EL_BS), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_GATHER: {
      const gather_args* A = (const gather_args*)dargs;
#define F(M)                                                                                                        \
  if (r2) hipLaunchKernelGGL((k_gather_rt<M, true>), g, dim3(256), 0, s, A, dboff, nr);                             \
  else hipLaunchKernelGGL((k_gather_rt<M, false>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_M(m, F);
#undef F
      break;
    }
    case RT_MAG_UPDATE: {
      const mag_update_args* A = (const mag_update_args*)dargs;
      if (mode != 1) return -2;  // plans hold SSP stages only
#define F(P, M)                                                                                                     \
  if (r2) hipLaunchKernelGGL((k_mag_update_rt<P, M, 1, MHD_MU_BS, true>), g, dim3(MHD_MU_BS), 0, s, A, dboff, nr);  \
  else hipLaunchKernelGGL((k_mag_update_rt<P, M, 1, MHD_MU_BS, false>), g, dim3(MHD_MU_BS), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_VEL_PREP: {
      const vel_prep_args* A = (const vel_prep_args*)dargs;
#define F(P) hipLaunchKernelGGL((k_vel_prep_rt<P>), g, dim3(MHD_PREP_BS), 0, s, A, dboff, nr)
      switch (h.key) { case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; case 4: F(4); break;
                       case 5: F(5); break; case 6: F(6); break; default: return -4; }
#undef F
      break;
    }
    case RT_VEL_SENSOR: {
      const vel_sensor_args* A = (const vel_sensor_args*)dargs;
#define F(P, M)                                                                                                     \
  if (r2) hipLaunchKernelGGL((k_vel_sensor_rt<P, M, true>), g, dim3(256), 0, s, A, dboff, nr);                      \
  else hipLaunchKernelGGL((k_vel_sensor_rt<P, M, false>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_VEL_PROJ: {
      const vel_proj_args* A = (const vel_proj_args*)dargs;
#define F(P)                                                                                                        \
  if (r2) hipLaunchKernelGGL((k_vel_proj_rt<P, MHD_VP_BS, true>), g, dim3(MHD_VP_BS), 0, s, A, dboff, nr);          \
  else hipLaunchKernelGGL((k_vel_proj_rt<P, MHD_VP_BS, false>), g, dim3(MHD_VP_BS), 0, s, A, dboff, nr)
      switch (p) { case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; case 4: F(4); break;
                   case 5: F(5); break; case 6: F(6); break; default: return -4; }
#undef F
      break;
    }
    case RT_B_STATS: {
      const B_stats_args* A = (const B_stats_args*)dargs;
#define F(M) hipLaunchKernelGGL((k_B_stats_rt<M>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_M(h.key, F);
#undef F
      break;
    }
    case RT_AR_TRACES: {
      const ar_traces_args* A = (const ar_traces_args*)dargs;
#define F(P, M) hipLaunchKernelGGL((k_ar_traces_rt<P, M>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_AR_ETA: {
      const ar_eta_args* A = (const ar_eta_args*)dargs;
#define F(P, M) hipLaunchKernelGGL((k_ar_eta_rt<P, M>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_PM(p, m, F);
#undef F
      break;
    }
    case RT_TO_PRIM:
      hipLaunchKernelGGL(k_to_primitive_rt, g, dim3(256), 0, s, (const prim_args*)dargs, dboff, nr);
      break;
    case RT_TO_CONS:
      hipLaunchKernelGGL(k_to_conservative_rt, g, dim3(256), 0, s, (const prim_args*)dargs, dboff, nr);
      break;
    default:
      return 1;  // not a kind of this file
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free magnetic residual: the same kernels as mhd25_rhs_magnetic, with the
// reconstructed J, E grids and the per-element loads in a fixed file-scope device array instead
// of the context's workspace, for callers that cannot allocate device memory.
// ---------------------------------------------------------------------------------------------
namespace {
constexpr long MHD_NOALLOC_DOUBLES = 4L << 20;  // 32 MiB per device
__device__ __align__(256) double scratch[MHD_NOALLOC_DOUBLES];
constexpr int MHD_MAX_DEVICES = 64;
double* g_scratch[MHD_MAX_DEVICES];  // device address of `scratch` on each device (set once)
std::mutex g_scratch_mu;
}  // namespace

// Resolves the device address of the scratch array on the current device, once per device (the
// name `scratch` in host code is only a stand-in, never a device address).  Called by mhd25_init.
int noalloc_setup(mhd25_ctx* c) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MHD_MAX_DEVICES) {
    c->err = "no-alloc setup: no current device";
    return -2;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return 0;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return -2;
  }
  g_scratch[dev] = (double*)ptr;
  return 0;
}

extern "C" int mhd25_rhs_magnetic_noalloc(mhd25_ctx* c, const double* rho, const double* u, const double* Bx,
                                          const double* By, const double* Bz, const double* eta, double* de,
                                          double* du, double* dBx, double* dBy, double* dBz) {
  if (!c || !rho || !u || !Bx || !By || !Bz || !de || !du || !dBx || !dBy || !dBz) return -1;
  const long K = c->mp.K, G = c->G;
  const long a = c->m + 2, b = c->m + 1;
  const long need = 6 * G + K * (2 * a * b + a * a);
  if (need > MHD_NOALLOC_DOUBLES) {
    c->err = "rhs_magnetic_noalloc: the mesh needs " + std::to_string(need * 8) + " bytes of scratch, above the " +
             std::to_string(MHD_NOALLOC_DOUBLES * 8) + "-byte limit";
    return -1;
  }
  int dev = 0;
  double* ws = nullptr;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < MHD_MAX_DEVICES) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ws = g_scratch[dev];
  }
  if (!ws) {
    c->err = "rhs_magnetic_noalloc: scratch not set up on the current device (create a context on it first)";
    return -2;
  }
  double* JE = ws;            // six grids: J_x, J_y, J_z, E_x, E_y, E_z
  double* loads = ws + 6 * G;  // every entry is written by the load kernels before the gathers read it
  const bool r2 = c->opt.reduced_2d2v != 0;
  if (const int r = reconstruct_JE_ws(c, u, Bx, By, Bz, eta, JE, r2, loads)) return r;
  MagIO io{};
  io.rho = rho; io.us = u; io.bxs = Bx; io.bys = By; io.bzs = Bz;
  io.jx = JE; io.jy = JE + G; io.jz = JE + 2 * G;
  io.ex = JE + 3 * G; io.ey = JE + 4 * G; io.ez = JE + 5 * G;
  io.eta = eta;
  io.oe = de; io.ou = du; io.obx = dBx; io.oby = dBy; io.obz = dBz;
  return mag_update(c, io, 0);
}
