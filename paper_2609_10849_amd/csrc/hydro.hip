// Hydrodynamic-subflow kernels for gfx950 (section "Hydrodynamic subflow: entropy-stable DGSEM").
//
// Mapping: one thread per GLL node, EB = 256 / (p+1)^2 elements per 256-thread block
// (wave64-friendly for every p).  The flux-differencing volume term uses the skew form
// sum_{r != i} S_ir F(U_i, U_r) (S = Q - Q^T), which equals eq. euler-volume-residual
// combined with the boundary corrections of eq. euler-nodal-index; each unordered pair of a
// line is evaluated once: the p(p+1)/2 pairs of a line are distributed cyclically over its
// p+1 nodes (node i owns pairs (i, i+d mod (p+1))), the owner accumulates its half in
// registers and hands the partner's half through LDS.  Reductions are in fixed order, so
// results are deterministic run to run.
#include <cfloat>

#include "common.h"
#include "xcd.h"
#include "ec_log.h"
#include "rsqrt.h"

namespace {

constexpr double EPSM = 2.220446049250313e-16;  // 2^-52

template <int P, int BS = 256>
struct Cfg {
  static constexpr int NP = P + 1, NN = NP * NP, EB = BS / NN, NT = EB * NN, ND = NP / 2;
};

struct Prim {
  double r, ux, uy, uz, b, lr, lb;
};

__device__ __forceinline__ Prim make_prim(const double U[5], double g) {
  Prim q;
  q.r = U[0];
  const double ir = rcp_refined(U[0]);  // rho > 0 on admissible states
  q.ux = U[1] * ir; q.uy = U[2] * ir; q.uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * q.ux + U[2] * q.uy + U[3] * q.uz));
  q.b = 0.5 * q.r * rcp_refined(p);  // p > 0 on admissible states
  q.lr = log_ec(q.r); q.lb = log_ec(q.b);
  return q;
}

// Logarithmic mean (eq. euler-chandrashekar-flux) as a fraction num/den from the node values
// a and their logarithms l.  Well separated (f^2 >= 1e-4 with f = (aR-aL)/(aR+aL)): (aR-aL)/(lR-lL).
// Near-equal: with x = (lR-lL)/2 = atanh f, the mean is (aL+aR) tanh(x) / (2x) = (aL+aR) / (2 x coth x),
// and 2 x coth x = 2 + y/6 - y^2/360 + y^3/15120 - ... in y = (lR-lL)^2 (the Laurent series of coth);
// there y < 4.1e-4, so the first omitted term is below 1e-19 relative.  The quotient is taken by the
// caller, which folds the three divisions of the flux into one reciprocal.
struct Frac {
  double n, d;
};
__device__ __forceinline__ Frac lmean_frac(double aL, double aR, double lL, double lR) {
  const double d = aR - aL, s = aR + aL, dl = lR - lL;
  const double y = dl * dl;
  const double pu = 2.0 + y * (1.0 / 6.0 - y * (1.0 / 360.0 - y * (1.0 / 15120.0)));
  const bool near = d * d < 1e-4 * (s * s);
  return Frac{near ? s : d, near ? pu : dl};
}

// Chandrashekar flux (eq. euler-chandrashekar-flux), energy in the form
// rho_log ud (gk/beta_log - |u|^2avg/2 + |avg u|^2) + p_hat ud with gk = 1/(2(g-1)).  rho_log = nR/dR,
// 1/beta_log = dB/nB and p_hat = (rhoL+rhoR)/(2(betaL+betaR)) share one reciprocal.
template <int D>
__device__ __forceinline__ void ecflux(const Prim& L, const Prim& R, double gk, double F[5]) {
  const Frac fr = lmean_frac(L.r, R.r, L.lr, R.lr);
  const Frac fb = lmean_frac(L.b, R.b, L.lb, R.lb);
  const double sb = L.b + R.b;
  const double t1 = fr.d * fb.n;
  const double Q = rcp_refined(t1 * sb);  // nonzero: each factor is a positive sum or a nonzero difference
  const double rl = fr.n * fb.n * sb * Q;
  const double ibl = fb.d * fr.d * sb * Q;
  const double ph = 0.5 * (L.r + R.r) * t1 * Q;
  const double uxa = 0.5 * (L.ux + R.ux), uya = 0.5 * (L.uy + R.uy), uza = 0.5 * (L.uz + R.uz);
  const double u2a = 0.5 * ((L.ux * L.ux + L.uy * L.uy + L.uz * L.uz) + (R.ux * R.ux + R.uy * R.uy + R.uz * R.uz));
  const double ud = D == 0 ? uxa : uya;
  const double f0 = rl * ud;
  F[0] = f0;
  F[1] = f0 * uxa + (D == 0 ? ph : 0.0);
  F[2] = f0 * uya + (D == 1 ? ph : 0.0);
  F[3] = f0 * uza;
  F[4] = f0 * (ibl * gk - 0.5 * u2a + (uxa * uxa + uya * uya + uza * uza)) + ph * ud;
}

// physical flux in direction D (0: x, 1: y, a run-time value so that x and y faces can share one
// code path), with the normal velocity and the sound speed
__device__ __forceinline__ void physflux(const double U[5], double g, int D, double F[5], double& ud, double& c) {
  const double ir = rcp_refined(U[0]);
  const double ux = U[1] * ir, uy = U[2] * ir, uz = U[3] * ir;
  const double p = (g - 1.0) * (U[4] - 0.5 * (U[1] * ux + U[2] * uy + U[3] * uz));
  ud = D == 0 ? ux : uy;
  F[0] = D == 0 ? U[1] : U[2];
  F[1] = U[1] * ud + (D == 0 ? p : 0.0);
  F[2] = U[2] * ud + (D == 1 ? p : 0.0);
  F[3] = U[3] * ud;
  F[4] = (U[4] + p) * ud;
  c = sqrt(g * p * ir);
}

// numerical interface flux in direction D between the element's own face value uo and the
// neighbour's un: LLF (eq. euler-lf-flux) or, for tests, the EC flux.  Both are symmetric in their
// two states except for the LLF jump U_R - U_L = sgn (un - uo) (sgn = +1 when the neighbour is the
// plus side), so no left/right copies are formed.
__device__ __forceinline__ void face_flux(const double uo[5], const double un[5], double sgn, double g, double gk,
                                          int D, int iface, double F[5]) {
  if (iface == 1) {
    Prim a = make_prim(uo, g), b = make_prim(un, g);
    if (D == 0) ecflux<0>(a, b, gk, F);
    else ecflux<1>(a, b, gk, F);
    return;
  }
  double Fo[5], Fn[5], udo, co, udn, cn;
  physflux(uo, g, D, Fo, udo, co);
  physflux(un, g, D, Fn, udn, cn);
  const double lam = fmax(fabs(udo) + co, fabs(udn) + cn);
#pragma unroll
  for (int c = 0; c < 5; ++c) F[c] = 0.5 * (Fo[c] + Fn[c]) - 0.5 * lam * (sgn * (un[c] - uo[c]));
}

// Face f = 2 D + side of element (ex, ey) (D 0: the x-normal faces, D 1: the y-normal faces; side 0
// is the face at -1) and the face node `line` on it: the neighbour element en across the face, the
// element's own face node qo and the neighbour's node qn at the same point (periodic mesh).
template <int P>
__device__ __forceinline__ void face_match(const MeshP& mp, int ex, int ey, int D, int side, int line, int& en,
                                           int& qo, int& qn) {
  constexpr int NP = P + 1;
  const int pos = side ? P : 0;
  qo = D == 0 ? line * NP + pos : pos * NP + line;
  qn = D == 0 ? line * NP + (P - pos) : (P - pos) * NP + line;
  en = D == 0 ? ey * mp.nx + wrap32(ex + (side ? 1 : -1), mp.nx) : wrap32(ey + (side ? 1 : -1), mp.ny) * mp.nx + ex;
}

// One direction of the volume part of L_E for the thread's node: owned pairs, incoming halves.
template <int P, int D, int BS>
__device__ __forceinline__ void volume_dir(const Prim& me, double acc[5], bool act, int el, int i, int j,
                                           double (*sp)[Cfg<P, BS>::EB * Cfg<P, BS>::NN], double* sb,
                                           const double* tS, const MeshP& mp) {
  using C = Cfg<P, BS>;
  constexpr int NP = C::NP, NN = C::NN, ND = C::ND;
  const int pos = D == 0 ? i : j, line = D == 0 ? j : i;
  const double sc = 2.0 * (D == 0 ? mp.rhx : mp.rhy);
  const double gk = mp.gk;
  // sb layout: [el][line][owner pos][dslot][5]
  double* sbl = sb + ((long)(el * NP + line) * NP) * ND * 5;
  if (act) {
#pragma unroll
    for (int d = 1; d <= ND; ++d) {
      if (2 * d == NP && pos >= NP / 2) continue;
      int r = pos + d;
      if (r >= NP) r -= NP;
      const int nr = el * NN + (D == 0 ? line * NP + r : r * NP + line);
      Prim o;
      o.r = sp[0][nr]; o.ux = sp[1][nr]; o.uy = sp[2][nr]; o.uz = sp[3][nr];
      o.b = sp[4][nr]; o.lr = sp[5][nr]; o.lb = sp[6][nr];
      double F[5];
      ecflux<D>(me, o, gk, F);
      const double ci = -sc * tS[pos * NP + r], cr = -sc * tS[r * NP + pos];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        acc[c] += ci * F[c];
        sbl[(pos * ND + (d - 1)) * 5 + c] = cr * F[c];
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
      for (int c = 0; c < 5; ++c) acc[c] += sbl[(o * ND + (d - 1)) * 5 + c];
    }
  }
  __syncthreads();
}

// Surface part of L_E: the element's 4 (p+1) interface fluxes as tasks f = (direction, side, line)
// with the direction a run-time value (x and y faces share one code path, so a wave runs the flux
// once), stored in sf = scr + el * 20 (p+1); then added at the face nodes.  The minus side of a face
// is the neighbour for side 0.  Every thread of the block must call this.
template <int P, int BS>
__device__ __forceinline__ void surface_terms(double acc[5], bool act, int el, int q, int i, int j, long e,
                                              const double* __restrict__ Us, long KN, double* scr,
                                              double (*sp)[Cfg<P, BS>::EB * Cfg<P, BS>::NN],
                                              const HydroTab* __restrict__ T, const MeshP& mp, int iface) {
  using C = Cfg<P, BS>;
  constexpr int NP = C::NP, NN = C::NN;
  double* sf = scr + el * 20 * NP;  // [f][5]
  const int tid = el * NN + q;
  if (act) {
    // the volume accumulators wait in the (now free) primitive rows, to keep registers for the fluxes
#pragma unroll
    for (int c = 0; c < 5; ++c) sp[c][tid] = acc[c];
    int ex, ey;
    elem_xy32(mp, (int)e, ex, ey);
    for (int f = q; f < 4 * NP; f += NN) {
      const int D = f / (2 * NP), side = (f / NP) & 1, line = f % NP;
      int en, qo, qn;
      face_match<P>(mp, ex, ey, D, side, line, en, qo, qn);
      const unsigned oo = ((unsigned)e * NN + qo) * 8u, on = ((unsigned)en * NN + qn) * 8u;
      double uo[5], un[5], F[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const auto r = node_rsrc(Us + c * KN, KN);
        uo[c] = bld(r, oo); un[c] = bld(r, on);
      }
      face_flux(uo, un, side ? 1.0 : -1.0, mp.gamma, mp.gk, D, iface, F);
      const double sc = 2.0 * (D == 0 ? mp.rhx : mp.rhy);
      const double s = side ? -(sc * rcp_refined(T->w[P])) : sc * rcp_refined(T->w[0]);
#pragma unroll
      for (int c = 0; c < 5; ++c) sf[f * 5 + c] = s * F[c];
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] = sp[c][tid];
    // face f = (D * 2 + side) * NP + line; x faces carry line j, y faces line i
    if (i == 0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += sf[(0 * NP + j) * 5 + c];
    }
    if (i == P) {
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += sf[(1 * NP + j) * 5 + c];
    }
    if (j == 0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += sf[(2 * NP + i) * 5 + c];
    }
    if (j == P) {
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += sf[(3 * NP + i) * 5 + c];
    }
  }
}

// Per-element sums (GLL weights, without |J_K|), minima and maxima of 5 fields held in LDS rows
// 0..4 of svf, plus the raw-average admissibility test (NaN-safe) from the five sums.  Two fixed-
// order levels: task (component, grid row) reduces its row into rs = sst + el * 15 NP (at least
// 15 (p+1) values per element, free LDS), then task (component, kind) combines the rows.  Rows
// 5..6 of svf (at least 5 values per element) take the sums; every thread of the block must call
// this.
template <class C>
__device__ __forceinline__ void element_stats(double* svf, double* sst, bool act, int el, int q, long e,
                                              double* __restrict__ stats, int* __restrict__ flag,
                                              const HydroTab* __restrict__ T, double g) {
  constexpr int NP = C::NP, NN = C::NN, S = C::EB * C::NN;
  double* rs = sst + el * 15 * NP;  // [component][kind][row]
  for (int t = q; act && t < 5 * NP; t += NN) {
    const int c = t / NP, r = t - c * NP;
    const double wr = T->w[r];
    double s = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double v = svf[c * S + el * NN + r * NP + i];
      s += (T->w[i] * wr) * v;
      mn = fmin(mn, v); mx = fmax(mx, v);
    }
    rs[(c * 3 + 0) * NP + r] = s;
    rs[(c * 3 + 1) * NP + r] = mn;
    rs[(c * 3 + 2) * NP + r] = mx;
  }
  __syncthreads();
  double* ssum = svf + 5 * S + el * 5;
  for (int t = q; act && t < 15; t += NN) {
    const int c = t / 3, kind = t - 3 * c;
    const double* v = rs + t * NP;
    double s = kind == 0 ? 0.0 : v[0];
#pragma unroll
    for (int r = kind == 0 ? 0 : 1; r < NP; ++r) s = kind == 0 ? s + v[r] : (kind == 1 ? fmin(s, v[r]) : fmax(s, v[r]));
    stats[(e * 5 + c) * 3 + kind] = s;
    if (kind == 0) ssum[c] = s;
  }
  if (!flag) return;
  __syncthreads();
  if (act && q == 0) {
    double a[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) a[c] = 0.25 * ssum[c];
    const double pb = (g - 1.0) * (a[4] - (a[1] * a[1] + a[2] * a[2] + a[3] * a[3]) / (2.0 * a[0]));
    if (!(a[0] > 0.0) || !(pb > 0.0)) atomicOr(flag, 1);
  }
}

// MODE 0: out = L_E(Us).  MODE 1: out = ca*Un + cb*(Us + tau*L_E(Us)) plus element statistics.
template <int P, int MODE, int BS>
__device__ __forceinline__ void hydro_stage_body(const double* __restrict__ Us, const double* __restrict__ Un,
                                                    double* __restrict__ out, double* __restrict__ stats,
                                                    int* __restrict__ flag, const HydroTab* __restrict__ T, MeshP mp,
                                                    double ca, double cb, double tau, int iface, long blk) {
  using C = Cfg<P, BS>;
  constexpr int NP = C::NP, NN = C::NN, EB = C::EB, ND = C::ND;
  __shared__ double sp[7][EB * NN];
  __shared__ double sb[EB * NP * NP * (ND > 0 ? ND : 1) * 5];
  __shared__ double tS[NP * NP];
  // scratch for the interface fluxes and the statistics' row partials (20 (p+1) values per
  // element): the flux hand-off buffer sb when it is large enough, else an array of its own
  constexpr bool SB_BIG = NP * (ND > 0 ? ND : 1) >= 4;
  __shared__ double sxt[SB_BIG ? 1 : EB * 20 * NP];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  if (tid < NP * NP) tS[tid] = T->Shat[tid / NP][tid % NP];
  if (MODE == 1) {  // skip stages after a rejected one; read once per block (other blocks may set it)
    if (tid == 0) sflag = __atomic_load_n(flag, __ATOMIC_RELAXED);
    __syncthreads();
    if (sflag) return;
  }
  const int el = tid / NN, q = tid - el * NN;
  const int i = q % NP, j = q / NP;
  const long e = blk * EB + el;
  const bool act = tid < C::NT && e < mp.K;
  const long KN = mp.K * NN;
  const unsigned no = ((unsigned)e * NN + q) * 8u;  // the node's byte offset in a component array
  double U[5], UNo[5], acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  Prim me{};
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) U[c] = bld(node_rsrc(Us + c * KN, KN), no);
    // U^n is issued early (it is only used at the end); the first stage (ca = 0) has no U^n term
    if (MODE == 1 && ca != 0.0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) UNo[c] = bld(node_rsrc(Un + c * KN, KN), no);
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) UNo[c] = 0.0;
    }
    me = make_prim(U, mp.gamma);
    sp[0][tid] = me.r; sp[1][tid] = me.ux; sp[2][tid] = me.uy; sp[3][tid] = me.uz;
    sp[4][tid] = me.b; sp[5][tid] = me.lr; sp[6][tid] = me.lb;
    // the SSP combine ca U^n + cb (U_s + tau L) is carried as (ca U^n + cb U_s) + cb tau L, so
    // that one state instead of two stays live through the flux phases
    if (MODE == 1) {
#pragma unroll
      for (int c = 0; c < 5; ++c) U[c] = ca * UNo[c] + cb * U[c];
    }
  }
  __syncthreads();
  volume_dir<P, 0, BS>(me, acc, act, el, i, j, sp, sb, tS, mp);
  volume_dir<P, 1, BS>(me, acc, act, el, i, j, sp, sb, tS, mp);
  double* scr = SB_BIG ? sb : sxt;
  surface_terms<P, BS>(acc, act, el, q, i, j, e, Us, KN, scr, sp, T, mp, iface);
  if (MODE == 0) {
    if (act) {
#pragma unroll
      for (int c = 0; c < 5; ++c) bst(node_rsrc(out + c * KN, KN), no, acc[c]);
    }
    return;
  }
  double Y[5];
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Y[c] = U[c] + (cb * tau) * acc[c];
      bst(node_rsrc(out + c * KN, KN), no, Y[c]);
      sp[c][tid] = Y[c];
    }
  }
  __syncthreads();
  element_stats<C>(&sp[0][0], scr, act, el, q, e, stats, flag, T, mp.gamma);
}

template <int P, int MODE, int BS>
__global__ __launch_bounds__(BS, P == 4 ? 4 : 1) void k_hydro_stage(const double* __restrict__ Us, const double* __restrict__ Un,
                                                    double* __restrict__ out, double* __restrict__ stats,
                                                    int* __restrict__ flag, const HydroTab* __restrict__ T, MeshP mp,
                                                    double ca, double cb, double tau, int iface) {
  hydro_stage_body<P, MODE, BS>(Us, Un, out, stats, flag, T, mp, ca, cb, tau, iface, (long)blockIdx.x);
}

struct hydro_stage_args {
  const double* Us;
  const double* Un;
  double* out;
  double* stats;
  int* flag;
  const HydroTab* T;
  MeshP mp;
  double ca;
  double cb;
  double tau;
  int iface;
};

template <int P, int MODE, int BS>
__global__ __launch_bounds__(BS, P == 4 ? 4 : 1) void k_hydro_stage_rt(const hydro_stage_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const hydro_stage_args& a = A[r];
  hydro_stage_body<P, MODE, BS>(gl(a.Us), gl(a.Un), gl(a.out), gl(a.stats), gl(a.flag), gl(a.T), a.mp, a.ca, a.cb, a.tau, a.iface, (long)blockIdx.x - boff[r]);
}

template <int P>
__global__ __launch_bounds__(256) void k_elem_stats(const double* __restrict__ Uin, double* __restrict__ stats,
                                                    int* __restrict__ flag, const HydroTab* __restrict__ T, MeshP mp) {
  using C = Cfg<P>;
  constexpr int NN = C::NN, EB = C::EB;
  __shared__ double sv[7][EB * NN];
  __shared__ double sst[EB * 15 * C::NP];
  const int tid = threadIdx.x;
  const int el = tid / NN, q = tid - el * NN;
  const long e = (long)blockIdx.x * EB + el;
  const bool act = tid < C::NT && e < mp.K;
  const long KN = mp.K * NN;
  if (act)
    for (int c = 0; c < 5; ++c) sv[c][tid] = Uin[c * KN + e * NN + q];
  __syncthreads();
  element_stats<Cfg<P>>(&sv[0][0], sst, act, el, q, e, stats, flag, T, mp.gamma);
}

// Element-average pressure helper
__device__ __forceinline__ double pres(const double* a, double g) {
  return (g - 1.0) * (a[4] - (a[1] * a[1] + a[2] * a[2] + a[3] * a[3]) / (2.0 * a[0]));
}
__device__ __forceinline__ double Sp(const double* a, double eps_r) {
  return fabs(a[4]) + (a[1] * a[1] + a[2] * a[2] + a[3] * a[3]) / (2.0 * fmax(a[0], eps_r));
}

// P = P_PP o P_OE on a raw stage (eq. euler-oe-map, eq. euler-pp-density, eq. euler-pp-pressure).
// The derivative jumps and the modal transforms run as line tasks: task (c, line) holds one grid
// line of component c in registers (five tasks per line index), so a line is read from LDS once
// per pass instead of once per output node; the 1D tables are read with uniform (scalar) loads.
// The element statistics of the raw stage (always formed before this map) give the element
// averages: the OE map keeps each element's mean, the (0, 0) Legendre mode.
template <int P, int BS>
__device__ __forceinline__ void hydro_oe_pp_body(const double* __restrict__ Ust, double* __restrict__ Uout,
                                                     const double* __restrict__ stats, const double* __restrict__ lines,
                                                     const double* __restrict__ glob, uint8_t* __restrict__ flags,
                                                     unsigned long long* __restrict__ counts,
                                                     const int* __restrict__ flag, const HydroTab* __restrict__ T,
                                                     MeshP mp, double tau, double sH, int do_oe, int do_pp,
                                                     double* __restrict__ rho_o, double* __restrict__ e_o,
                                                     double* __restrict__ u_o, long blk) {
  using C = Cfg<P, BS>;
  constexpr int NP = C::NP, NN = C::NN, EB = C::EB, NL = 5 * NP;
  __shared__ double su[5][EB * NN];
  __shared__ double st[10][EB * NN];
  __shared__ double ssig0[EB][NP], ssig1[EB][NP], ssg[EB][5][NP];
  __shared__ double sD[EB][NP], samp[EB][2][5], srow[EB][3][NP];
  __shared__ int scst[EB][5];
  if (flag && *flag) return;
  const int tid = threadIdx.x;
  const int el = tid / NN, q = tid - el * NN;
  const long e = blk * EB + el;
  const bool act = tid < C::NT && e < mp.K;
  const long KN = mp.K * NN;
  const unsigned no = ((unsigned)e * NN + q) * 8u;  // the node's byte offset in a component array
  const double g = mp.gamma;
  int ex, ey;
  elem_xy32(mp, act ? (int)e : 0, ex, ey);
  // grid line ln of direction D (D = 0: row, index along x; D = 1: column), position k on it
  auto nodeof = [](int D, int ln, int k) { return D == 0 ? ln * NP + k : k * NP + ln; };
  double U[5], a[5];
  // the four neighbours' nodes (x minus, x plus, y minus, y plus) are loaded into registers up
  // front with the element's own, so that their latency overlaps the amplitude and x phases; they
  // go to LDS when their direction comes
  double nb[4][5];
  if (act && do_oe) {
    const int nbe[4] = {ey * mp.nx + wrap32(ex - 1, mp.nx), ey * mp.nx + wrap32(ex + 1, mp.nx),
                        wrap32(ey - 1, mp.ny) * mp.nx + ex, wrap32(ey + 1, mp.ny) * mp.nx + ex};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const unsigned on = ((unsigned)nbe[s] * NN + q) * 8u;
#pragma unroll
      for (int c = 0; c < 5; ++c) nb[s][c] = bld(node_rsrc(Ust + c * KN, KN), on);
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) { U[c] = bld(node_rsrc(Ust + c * KN, KN), no); su[c][tid] = U[c]; }
#pragma unroll
    for (int c = 0; c < 5; ++c) a[c] = 0.25 * stats[(e * 5 + c) * 3];
  }
  double rmin = act ? stats[(e * 5) * 3 + 1] : DBL_MAX;  // raw-stage density minimum (no OE)
  __syncthreads();
  if (do_oe) {
    // global and cross-line amplitudes (eq. euler-oe-amplitude), one task per component
    for (int c = q; act && c < 5; c += NN) {
      const double gs = glob[c * 3 + 0], gmn = glob[c * 3 + 1], gmx = glob[c * 3 + 2];
      const double gm = gs * mp.r4K;
      const double dOm = fmax(gmx - gm, gm - gmn);
      // constant to roundoff: the nodal values agree to 2^10 ulps of the field's size (exact test)
      scst[el][c] = gmx - gmn <= 1024.0 * EPSM * fmax(fabs(gmx), fabs(gmn)) ? 1 : 0;
      const double* rl = lines + (ey * 5 + c) * 3;
      const double* cl = lines + ((mp.ny + ex) * 5 + c) * 3;
      const double rm = rl[0] * mp.r4nx, cm = cl[0] * mp.r4ny;
      samp[el][0][c] = fmax(fmax(rl[2] - rm, rm - rl[1]), 1e-6 * dOm);
      samp[el][1][c] = fmax(fmax(cl[2] - cm, cm - cl[1]), 1e-6 * dOm);
    }
#pragma unroll
    for (int D = 0; D < 2; ++D) {
      // neighbours across the two faces normal to direction D, staged in st rows 0..9
      // (row c: minus-side neighbour, row 5 + c: plus-side neighbour)
      if (act) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          st[c][tid] = nb[2 * D][c];
          st[5 + c][tid] = nb[2 * D + 1][c];
        }
      }
      if (D == 1 && act && q < NP) {  // direction-0 sigma: maximum over the components
        double sg = 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) sg = fmax(sg, ssg[el][c][q]);
        ssig0[el][q] = sg;
      }
      __syncthreads();
      // normal-jump contributions (eq. euler-oe-jump) of line ln of component c: the r-th
      // derivatives at both faces of the element and of its neighbours.  The squared, weighted
      // jumps of derivative order r overwrite the task's own staged slots (position r on the line)
      for (int t = q; act && t < NL; t += NN) {
        const int ln = t / 5, c = t - ln * 5;  // component fastest (fewer LDS bank conflicts)
        double own[NP], mn[NP], pl[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int n = el * NN + nodeof(D, ln, k);
          own[k] = su[c][n]; mn[k] = st[c][n]; pl[k] = st[5 + c][n];
        }
        const double wl = 0.5 * T->w[ln];
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          double ja = 0.0, jd = 0.0, jb = 0.0, jc = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            // the +1 row from the -1 row: on the symmetric GLL nodes d^r l_k (+1) = (-1)^r d^r l_{p-k} (-1),
            // which the tables hold bit for bit, so one table stays in scalar registers instead of two
            const double d0 = T->Dr0[r][k], dp = (r & 1) ? -T->Dr0[r][P - k] : T->Dr0[r][P - k];
            ja += d0 * own[k];
            jd += dp * own[k];
            jb += dp * mn[k];
            jc += d0 * pl[k];
          }
          const double jm = ja - jb, jp = jc - jd;
          const int n = el * NN + nodeof(D, ln, r);
          st[c][n] = wl * jm * jm;
          st[5 + c][n] = wl * jp * jp;
        }
      }
      __syncthreads();
      // sigma (eq. euler-oe-sigma): task (r, c) sums its squared jumps over the lines
      {
        double Dsh = 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) Dsh = act ? fmax(Dsh, samp[el][D][c]) : 0.0;
        for (int t = q; act && t < 5 * NP; t += NN) {
          const int rr = t / 5, c = t - rr * 5;
          double v = 0.0;
          if (Dsh > 0.0 && !scst[el][c]) {
            double sm = 0.0, spp = 0.0;
            for (int l = 0; l < NP; ++l) {
              const int n = el * NN + nodeof(D, l, rr);
              sm += st[c][n];
              spp += st[5 + c][n];
            }
            v = T->fr[rr] * (sqrt(sm) + sqrt(spp)) / Dsh;
          }
          ssg[el][c][rr] = v;  // direction 0's values are reduced before direction 1 writes
        }
      }
      __syncthreads();
    }
    // modal damping with line tasks: x transform of each row, then per column the y transform,
    // the shell factors and the inverse y transform, then the inverse x transform of each row.
    // On the symmetric GLL nodes Tf[a][k] = (-1)^a Tf[a][p-k] and V[k][a] = (-1)^a V[p-k][a], bit for
    // bit in the tables, so only the entries with k <= p/2 are read (fewer scalar registers).
    auto tf = [&](int a, int k) {
      return k <= P / 2 ? T->Tf[a][k] : ((a & 1) ? -T->Tf[a][P - k] : T->Tf[a][P - k]);
    };
    auto vt = [&](int k, int a) {
      return k <= P / 2 ? T->V[k][a] : ((a & 1) ? -T->V[P - k][a] : T->V[P - k][a]);
    };
    for (int t = q; act && t < NL; t += NN) {
      const int ln = t / 5, c = t - ln * 5;  // component fastest (fewer LDS bank conflicts)
      double v[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = su[c][el * NN + ln * NP + k];
#pragma unroll
      for (int aa = 0; aa < NP; ++aa) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) s += tf(aa, k) * v[k];
        st[c][el * NN + ln * NP + aa] = s;  // [row][x mode]
      }
    }
    if (act && q < NP) {  // direction-1 sigma: maximum over the components
      double sg = 0.0;
#pragma unroll
      for (int c = 0; c < 5; ++c) sg = fmax(sg, ssg[el][c][q]);
      ssig1[el][q] = sg;
    }
    __syncthreads();
    // shell damping factors (eq. euler-oe-map): D_l = exp(-s tau (lx sum_{r<=l} sigma_x,r + ...)),
    // with one reciprocal of the mean density
    if (act && q <= P) {
      if (q == 0) {
        sD[el][0] = 1.0;
      } else {
        const double ir0 = 1.0 / a[0];
        const double pa = (g - 1.0) * (a[4] - 0.5 * (a[1] * a[1] + a[2] * a[2] + a[3] * a[3]) * ir0);
        const double ck = sqrt(g * pa * ir0);
        const double lx = (2.0 * P + 1.0) * (fabs(a[1] * ir0) + ck) * mp.rhx;
        const double ly = (2.0 * P + 1.0) * (fabs(a[2] * ir0) + ck) * mp.rhy;
        double sx = 0.0, sy = 0.0;
        for (int r = 0; r <= q; ++r) { sx += ssig0[el][r]; sy += ssig1[el][r]; }
        sD[el][q] = exp(-sH * tau * (lx * sx + ly * sy));
      }
    }
    __syncthreads();
    for (int t = q; act && t < NL; t += NN) {
      const int aa = t / 5, c = t - aa * 5;
      double v[NP], cb[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = st[c][el * NN + k * NP + aa];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) s += tf(b, k) * v[k];
        cb[b] = sD[el][aa > b ? aa : b] * s;  // coefficient (x mode aa, y mode b), damped
      }
#pragma unroll
      for (int jj = 0; jj < NP; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NP; ++b) s += vt(jj, b) * cb[b];
        st[c][el * NN + jj * NP + aa] = s;  // [row][x mode]
      }
    }
    __syncthreads();
    for (int t = q; act && t < NL; t += NN) {
      const int ln = t / 5, c = t - ln * 5;  // component fastest (fewer LDS bank conflicts)
      double v[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = st[c][el * NN + ln * NP + k];
      double mn = DBL_MAX;
#pragma unroll
      for (int ii = 0; ii < NP; ++ii) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) s += vt(ii, k) * v[k];
        su[c][el * NN + ln * NP + ii] = s;
        mn = fmin(mn, s);
      }
      if (c == 0) srow[el][0][ln] = mn;  // row minimum of the damped density
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 5; ++c) U[c] = su[c][tid];
      rmin = DBL_MAX;
#pragma unroll
      for (int l = 0; l < NP; ++l) rmin = fmin(rmin, srow[el][0][l]);
    }
  }
  uint8_t f = 0;
  if (do_pp) {
    // positivity scaling: the S_p and pressure extrema are reduced per row (NP tasks per
    // element), then over the rows by every thread
    const double eps_r = 64.0 * EPSM;
    const bool collapse_r = !(a[0] > eps_r);
    double thr = 1.0;
    if (act && !collapse_r && rmin < eps_r) {
      thr = fmin(1.0, fmax(0.0, (a[0] - eps_r) / (a[0] - rmin)));
      f |= 1;
      U[0] = a[0] + thr * (U[0] - a[0]);  // density-limited state of this node
    }
    if (act) {
      st[0][tid] = Sp(U, eps_r);
      st[1][tid] = pres(U, g);
    }
    __syncthreads();
    for (int t = q; act && t < NP; t += NN) {
      double S = 0.0, pm = DBL_MAX;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        S = fmax(S, st[0][el * NN + t * NP + k]);
        pm = fmin(pm, st[1][el * NN + t * NP + k]);
      }
      srow[el][1][t] = S;
      srow[el][2][t] = pm;
    }
    __syncthreads();
    if (act && !collapse_r) {
      double S = Sp(a, eps_r), pmin = DBL_MAX;
#pragma unroll
      for (int l = 0; l < NP; ++l) { S = fmax(S, srow[el][1][l]); pmin = fmin(pmin, srow[el][2][l]); }
      const double eps_p = fmax(64.0 * EPSM, 8192.0 * EPSM * S);
      const double pb = pres(a, g);
      if (pb <= eps_p) {
        f |= 4;
#pragma unroll
        for (int c = 0; c < 5; ++c) U[c] = a[c];
      } else if (pmin < eps_p) {
        const double thp = fmin(1.0, fmax(0.0, (pb - eps_p) / (pb - pmin)));
        f |= 2;
#pragma unroll
        for (int c = 0; c < 5; ++c) U[c] = a[c] + thp * (U[c] - a[c]);
      }
    } else if (act && collapse_r) {
      f = 4;
#pragma unroll
      for (int c = 0; c < 5; ++c) U[c] = a[c];
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) bst(node_rsrc(Uout + c * KN, KN), no, U[c]);
    if (rho_o) {  // primitive copy for the magnetic substep (the conversion's arithmetic)
      const double r = U[0], ux = U[1] / r, uy = U[2] / r, uz = U[3] / r;
      bst(node_rsrc(rho_o, KN), no, r);
      bst(node_rsrc(u_o, KN), no, ux); bst(node_rsrc(u_o + KN, KN), no, uy); bst(node_rsrc(u_o + 2 * KN, KN), no, uz);
      bst(node_rsrc(e_o, KN), no, (U[4] - 0.5 * r * (ux * ux + uy * uy + uz * uz)) / r);
    }
    if (q == 0) {
      if (flags) flags[e] = f;
      if (counts && f) {
        if (f & 1) atomicAdd(&counts[0], 1ull);
        if (f & 2) atomicAdd(&counts[1], 1ull);
        if (f & 4) atomicAdd(&counts[2], 1ull);
      }
    }
  }
}

template <int P, int BS>
__global__ __launch_bounds__(BS) void k_hydro_oe_pp(const double* __restrict__ Ust, double* __restrict__ Uout,
                                                     const double* __restrict__ stats, const double* __restrict__ lines,
                                                     const double* __restrict__ glob, uint8_t* __restrict__ flags,
                                                     unsigned long long* __restrict__ counts,
                                                     const int* __restrict__ flag, const HydroTab* __restrict__ T,
                                                     MeshP mp, double tau, double sH, int do_oe, int do_pp,
                                                     double* __restrict__ rho_o, double* __restrict__ e_o,
                                                     double* __restrict__ u_o) {
  hydro_oe_pp_body<P, BS>(Ust, Uout, stats, lines, glob, flags, counts, flag, T, mp, tau, sH, do_oe, do_pp, rho_o, e_o, u_o, xcd_block());
}

struct hydro_oe_pp_args {
  const double* Ust;
  double* Uout;
  const double* stats;
  const double* lines;
  const double* glob;
  uint8_t* flags;
  unsigned long long* counts;
  const int* flag;
  const HydroTab* T;
  MeshP mp;
  double tau;
  double sH;
  int do_oe;
  int do_pp;
  double* rho_o;
  double* e_o;
  double* u_o;
};

template <int P, int BS>
__global__ __launch_bounds__(BS) void k_hydro_oe_pp_rt(const hydro_oe_pp_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const hydro_oe_pp_args& a = A[r];
  hydro_oe_pp_body<P, BS>(gl(a.Ust), gl(a.Uout), gl(a.stats), gl(a.lines), gl(a.glob), gl(a.flags), gl(a.counts), gl(a.flag), gl(a.T), a.mp, a.tau, a.sH, a.do_oe, a.do_pp, gl(a.rho_o), gl(a.e_o), gl(a.u_o), (long)blockIdx.x - boff[r]);
}

// Connectivity export: nbr[K][4] (left, right, bottom, top neighbour) and the face map
// fmap[K][4][p+1] (the neighbour node e' (p+1)^2 + q' matched to each own face node), formed with the
// same face_match the stage kernel uses.  One thread per (element, face).
template <int P>
__global__ __launch_bounds__(256) void k_face_map(int32_t* __restrict__ nbr, int32_t* __restrict__ fmap, MeshP mp) {
  constexpr int NP = P + 1, NN = NP * NP;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * mp.K) return;
  const long e = t >> 2;
  const int f = (int)(t & 3), D = f >> 1, side = f & 1;
  int ex, ey;
  elem_xy32(mp, (int)e, ex, ey);
  int en = 0;
  for (int line = 0; line < NP; ++line) {
    int qo, qn;
    face_match<P>(mp, ex, ey, D, side, line, en, qo, qn);
    if (fmap) fmap[t * NP + line] = en * NN + qn;
  }
  nbr[t] = en;
}

// Entry copy of a conservative state with the admissibility test of every node: all five values
// finite, rho > 0 and p > 0 (the admissible set of section "Conservative ideal MHD").  A failing node
// sets bit 1 of flag[1].  One thread per node.
__device__ __forceinline__ void snap_check_node(const double* __restrict__ U, double* __restrict__ snap, long KN,
                                                double g, int* __restrict__ flag, long n) {
  double v[5];
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    v[c] = U[c * KN + n];
    snap[c * KN + n] = v[c];
    fin = fin && fabs(v[c]) <= DBL_MAX;
  }
  const double p = (g - 1.0) * (v[4] - (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / (2.0 * v[0]));
  if (!fin || !(v[0] > 0.0) || !(p > 0.0)) atomicOr(flag + 1, 2);
}

__global__ __launch_bounds__(256) void k_snap_check_U(const double* __restrict__ U, double* __restrict__ snap, long KN,
                                                      double g, int* __restrict__ flag) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < KN; n += (long)gridDim.x * blockDim.x)
    snap_check_node(U, snap, KN, g, flag, n);
}

// entry copy with a finiteness test (magnetic grids); a non-finite value sets bit 1 of flag[1]
__global__ __launch_bounds__(256) void k_copy_check(const double* __restrict__ a, double* __restrict__ b, long n,
                                                    int* __restrict__ flag) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const double v = a[k];
    b[k] = v;
    if (!(fabs(v) <= DBL_MAX)) atomicOr(flag + 1, 2);
  }
}

}  // namespace

// Row / column reduction of per-element statistics [K][nc][3] (sum, min, max), nc <= 5, fixed
// order.  Blocks 0..ny-1 reduce one element row each: thread t takes elements t, t+256, ... of
// the row and reads each element's nc*3 values as one contiguous record.  Blocks ny.. reduce
// LRC adjacent element columns each: thread (column j, phase p) takes rows p, p+LRP, ... of
// column j, so a wave reads adjacent elements of one row.  Partial results are combined in LDS
// by a fixed tree.
constexpr int LRC = 8, LRP = 256 / LRC;

// A row reduces its first rx elements and a column its first ry (the whole mesh on a periodic
// domain; the box of a mirror-walled mesh, whose other elements are mirror images: every row's and
// column's statistics are then those of the box's own, up to the sign of an odd field).
template <int NC>
__device__ __forceinline__ void line_reduce_body(const double* __restrict__ stats, double* __restrict__ lines,
                                                     int nx, int ny, int rx, int ry, const int* __restrict__ flag,
                                                     long blk) {
  constexpr int nc = NC;  // components per element record (compile-time, so that no load waits on a branch)
  __shared__ double red[15][256];
  if (flag && *flag) return;
  const int b = blk, t = threadIdx.x;
  const int nv = nc * 3;
  double v[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) v[k] = (k % 3 == 0) ? 0.0 : (k % 3 == 1 ? DBL_MAX : -DBL_MAX);
  auto take = [&](long e) {
    const double* st = stats + e * nv;
#pragma unroll
    for (int c = 0; c < 5; ++c)
      if (c < nc) {
        v[3 * c] += st[3 * c];
        v[3 * c + 1] = fmin(v[3 * c + 1], st[3 * c + 1]);
        v[3 * c + 2] = fmax(v[3 * c + 2], st[3 * c + 2]);
      }
  };
  // (unrolled by 4 so that four records' loads are in flight at once; the accumulation order, and so
  // every result bit, is that of the plain loop)
  if (b < ny) {
#pragma unroll 4
    for (int k = t; k < rx; k += 256) take((long)b * nx + k);
  } else {
    const int col = (b - ny) * LRC + t % LRC, ph = t / LRC;
    if (col < nx)
#pragma unroll 4
      for (int r = ph; r < ry; r += LRP) take((long)r * nx + col);
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) red[k][t] = v[k];
  __syncthreads();
  // rows: tree over all 256 threads; columns: tree over the LRP phases of each column
  const int lo = b < ny ? 1 : LRC;
  for (int w = 128; w >= lo; w >>= 1) {
    if (t < w)
      for (int c = 0; c < nc; ++c) {
        red[3 * c][t] += red[3 * c][t + w];
        red[3 * c + 1][t] = fmin(red[3 * c + 1][t], red[3 * c + 1][t + w]);
        red[3 * c + 2][t] = fmax(red[3 * c + 2][t], red[3 * c + 2][t + w]);
      }
    __syncthreads();
  }
  if (b < ny) {
    if (t < nv) lines[(long)b * nv + t] = red[t][0];
  } else if (t < LRC * nv) {
    const int j = t % LRC, k = t / LRC, col = (b - ny) * LRC + j;
    if (col < nx) lines[((long)ny + col) * nv + k] = red[k][j];
  }
}

template <int NC>
__global__ __launch_bounds__(256) void k_line_reduce(const double* __restrict__ stats, double* __restrict__ lines,
                                                     int nx, int ny, int rx, int ry, const int* __restrict__ flag) {
  line_reduce_body<NC>(stats, lines, nx, ny, rx, ry, flag, (long)blockIdx.x);
}

struct line_reduce_args {
  const double* stats;
  double* lines;
  int nx;
  int ny;
  int rx;
  int ry;
  const int* flag;
};

template <int NC>
__global__ __launch_bounds__(256) void k_line_reduce_rt(const line_reduce_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const line_reduce_args& a = A[r];
  line_reduce_body<NC>(gl(a.stats), gl(a.lines), a.nx, a.ny, a.rx, a.ry, gl(a.flag), (long)blockIdx.x - boff[r]);
}

// Global reduction of the first `n` line results (the rows of the periodic mesh or of the box) into glob[nc][3]: all NC components in
// one tree (each component's accumulation order is that of its own tree), so the block passes
// eight barriers instead of eight per component.
template <int NC>
__device__ __forceinline__ void global_reduce_body(const double* __restrict__ lines, double* __restrict__ glob,
                                                       int n, const int* __restrict__ flag, long blk) {
  __shared__ double red[3 * NC][256];
  if (flag && *flag) return;
  const int t = threadIdx.x;
  double v[3 * NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) { v[3 * c] = 0.0; v[3 * c + 1] = DBL_MAX; v[3 * c + 2] = -DBL_MAX; }
  for (int k = t; k < n; k += 256) {
    const double* st = lines + (long)k * NC * 3;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      v[3 * c] += st[3 * c];
      v[3 * c + 1] = fmin(v[3 * c + 1], st[3 * c + 1]);
      v[3 * c + 2] = fmax(v[3 * c + 2], st[3 * c + 2]);
    }
  }
#pragma unroll
  for (int x = 0; x < 3 * NC; ++x) red[x][t] = v[x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        red[3 * c][t] += red[3 * c][t + w];
        red[3 * c + 1][t] = fmin(red[3 * c + 1][t], red[3 * c + 1][t + w]);
        red[3 * c + 2][t] = fmax(red[3 * c + 2][t], red[3 * c + 2][t + w]);
      }
    __syncthreads();
  }
  if (t < 3 * NC) glob[t] = red[t][0];
}

template <int NC>
__global__ __launch_bounds__(256) void k_global_reduce(const double* __restrict__ lines, double* __restrict__ glob,
                                                       int n, const int* __restrict__ flag) {
  global_reduce_body<NC>(lines, glob, n, flag, (long)blockIdx.x);
}

struct global_reduce_args {
  const double* lines;
  double* glob;
  int n;
  const int* flag;
};

template <int NC>
__global__ __launch_bounds__(256) void k_global_reduce_rt(const global_reduce_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const global_reduce_args& a = A[r];
  global_reduce_body<NC>(gl(a.lines), gl(a.glob), a.n, gl(a.flag), (long)blockIdx.x - boff[r]);
}

// argument structs of the small and flat kernels for run-table launches
struct reset_args {
  int* flag;
  unsigned long long* counts;
  int clear_input;
};
struct copy_args {
  const double* a;
  double* b;
  long n;
  int* flag;  // non-null: finiteness test into flag[1]
};
struct snap_args {
  const double* U;
  double* snap;
  long KN;
  double g;
  int* flag;
};

// flag[0]: the attempt's reject word (bit 0: an inadmissible raw average), which the stage kernels
// test to skip the rest of a failed attempt; flag[1]: the entry check's word (bit 1: an inadmissible
// input), cleared at entry and copied into flag[0] at the start of every attempt so that an attempt
// on an inadmissible input does no work.
__global__ void k_reset_attempt(int* flag, unsigned long long* counts, int clear_input) {
  if (threadIdx.x == 0) {
    if (clear_input) flag[1] = 0;
    flag[0] = flag[1];
    counts[0] = 0; counts[1] = 0; counts[2] = 0;
  }
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, long n) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) b[k] = a[k];
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
#define DISPATCH_P(p, F) \
  switch (p) { case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; \
               case 4: F(4); break; case 5: F(5); break; case 6: F(6); break; default: return -4; }

hipEvent_t* timing_slot(mhd25_ctx* c, int kid);
static int eb_of(int p) { return 256 / ((p + 1) * (p + 1)); }
// threads per block of the hydro stage kernel: the tuned value if set, else 128 up to N = 4 (all
// lanes but three carry nodes, and the kernel fits 128 VGPRs without spills) and 256 above (fewer
// idle lanes for (N+1)^2 = 36, 49)
static int stage_block(const mhd25_ctx* c) {
  if (c->hydro_bs == 128 || c->hydro_bs == 256) return c->hydro_bs;
  return c->p <= 4 ? 128 : 256;
}

static int check(mhd25_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) { c->err = std::string(what) + ": " + hipGetErrorString(e); return -2; }
  return 0;
}

// row and column reductions of nc-component element records (nc = 1..5), then the global one
static int launch_reductions(mhd25_ctx* c, const double* stats, int nc, const int* flag) {
  const dim3 grid(c->mp.ny + (c->mp.nx + LRC - 1) / LRC);
  if (c->rec) {
    rt_record(c, RT_LINE_REDUCE, nc, grid.x,
              line_reduce_args{stats, c->lines, c->mp.nx, c->mp.ny, c->mp.bx, c->mp.by, flag});
    rt_record(c, RT_GLOBAL_REDUCE, nc, 1, global_reduce_args{c->lines, c->glob, c->mp.by, flag});
    return 0;
  }
#define LR(NC)                                                                                                    \
  hipLaunchKernelGGL((k_line_reduce<NC>), grid, dim3(256), 0, c->stream, stats, c->lines, c->mp.nx, c->mp.ny,    \
                     c->mp.bx, c->mp.by, flag);                                                                   \
  hipLaunchKernelGGL((k_global_reduce<NC>), dim3(1), dim3(256), 0, c->stream, c->lines, c->glob, c->mp.by, flag)
  switch (nc) { case 1: LR(1); break; case 2: LR(2); break; case 3: LR(3); break; case 4: LR(4); break;
                case 5: LR(5); break; default: c->err = "line reduction: unsupported component count"; return -2; }
#undef LR
  return 0;
}

int hydro_rhs(mhd25_ctx* c, const double* U, double* dU) {
  const int bs = stage_block(c);
  const int eb = bs / ((c->p + 1) * (c->p + 1));
  const long blocks = (c->mp.K + eb - 1) / eb;
#define L0(P)                                                                                                      \
  if (bs == 128) hipLaunchKernelGGL((k_hydro_stage<P, 0, 128>), dim3(blocks), dim3(128), 0, c->stream, U, U, dU,  \
                                    nullptr, nullptr, c->d_ht, c->mp, 0.0, 1.0, 0.0, c->opt.iface_flux);          \
  else hipLaunchKernelGGL((k_hydro_stage<P, 0, 256>), dim3(blocks), dim3(256), 0, c->stream, U, U, dU, nullptr,    \
                          nullptr, c->d_ht, c->mp, 0.0, 1.0, 0.0, c->opt.iface_flux)
  DISPATCH_P(c->p, L0);
#undef L0
  return check(c, hipGetLastError(), "rhs_hydro launch");
}

// raw stage + statistics + line/global reductions
int hydro_stage_a(mhd25_ctx* c, const double* Us, const double* Un, double* Ust, double ca, double cb, double tau) {
  const int bs = stage_block(c);
  const int eb = bs / ((c->p + 1) * (c->p + 1));
  const long blocks = (c->mp.K + eb - 1) / eb;
  if (c->rec) {
    rt_record(c, RT_HYDRO_STAGE, c->p * 1000 + bs, blocks,
              hydro_stage_args{Us, Un, Ust, c->stats, c->d_flag, c->d_ht, c->mp, ca, cb, tau, c->opt.iface_flux});
    return launch_reductions(c, c->stats, 5, c->d_flag);
  }
  hipEvent_t* ev = c->timing ? timing_slot(c, 0) : nullptr;
  if (ev) hipEventRecord(ev[0], c->stream);
#define L1(P)                                                                                                      \
  if (bs == 128) hipLaunchKernelGGL((k_hydro_stage<P, 1, 128>), dim3(blocks), dim3(128), 0, c->stream, Us, Un, Ust, \
                                    c->stats, c->d_flag, c->d_ht, c->mp, ca, cb, tau, c->opt.iface_flux);          \
  else hipLaunchKernelGGL((k_hydro_stage<P, 1, 256>), dim3(blocks), dim3(256), 0, c->stream, Us, Un, Ust, c->stats, \
                          c->d_flag, c->d_ht, c->mp, ca, cb, tau, c->opt.iface_flux)
  DISPATCH_P(c->p, L1);
#undef L1
  if (ev) hipEventRecord(ev[1], c->stream);
  int r = check(c, hipGetLastError(), "hydro stage launch");
  if (r) return r;
  if (const int rl = launch_reductions(c, c->stats, 5, c->d_flag)) return rl;
  return check(c, hipGetLastError(), "reduce launch");
}

int line_global_reduce(mhd25_ctx* c, const double* stats, int nc, const int* flag) {
  if (const int r = launch_reductions(c, stats, nc, flag)) return r;
  return check(c, hipGetLastError(), "reduce launch");
}

int hydro_stats_only(mhd25_ctx* c, const double* U, int* flag) {
  const long blocks = (c->mp.K + eb_of(c->p) - 1) / eb_of(c->p);
#define LS(P) hipLaunchKernelGGL((k_elem_stats<P>), dim3(blocks), dim3(256), 0, c->stream, U, c->stats, flag, c->d_ht, c->mp)
  DISPATCH_P(c->p, LS);
#undef LS
  if (const int rl = launch_reductions(c, c->stats, 5, nullptr)) return rl;
  return check(c, hipGetLastError(), "stats launch");
}

// threads per block of the OE/PP map: its LDS use (about 35 KB at N = 4 with 256 threads) caps a CU
// at 4 such blocks, 4 waves per SIMD; with 128 threads the registers allow 5 waves per SIMD, which
// measured 10 % faster on the 1024^2, N = 4 workload
#ifndef MHD_OE_BS
#define MHD_OE_BS 128
#endif

// rho_o, e_o, u_o: optional primitive outputs (all null or all set)
int hydro_stage_b(mhd25_ctx* c, const double* Ust, double* Uout, double tau, const int* flag, double* rho_o,
                  double* e_o, double* u_o) {
  constexpr int BS = MHD_OE_BS;
  const int eb = BS / ((c->p + 1) * (c->p + 1));
  const long blocks = (c->mp.K + eb - 1) / eb;
  if (c->rec) {
    rt_record(c, RT_OE_PP, c->p, blocks,
              hydro_oe_pp_args{Ust, Uout, c->stats, c->lines, c->glob, c->d_flags, c->d_counts, flag, c->d_ht, c->mp,
                               tau, c->opt.s_H, c->opt.oe_hydro, c->opt.pp, rho_o, e_o, u_o});
    return 0;
  }
  hipEvent_t* ev = c->timing ? timing_slot(c, 1) : nullptr;
  if (ev) hipEventRecord(ev[0], c->stream);
#define LB(P) hipLaunchKernelGGL((k_hydro_oe_pp<P, BS>), dim3(blocks), dim3(BS), 0, c->stream, Ust, Uout, c->stats, \
                                 c->lines, c->glob, c->d_flags, c->d_counts, flag, c->d_ht, c->mp, tau, c->opt.s_H, \
                                 c->opt.oe_hydro, c->opt.pp, rho_o, e_o, u_o)
  DISPATCH_P(c->p, LB);
#undef LB
  if (ev) hipEventRecord(ev[1], c->stream);
  return check(c, hipGetLastError(), "stage map launch");
}

int reset_attempt(mhd25_ctx* c) {
  if (c->rec) { rt_record(c, RT_RESET, 0, 1, reset_args{c->d_flag, c->d_counts, 0}); return 0; }
  hipLaunchKernelGGL(k_reset_attempt, dim3(1), dim3(64), 0, c->stream, c->d_flag, c->d_counts, 0);
  return check(c, hipGetLastError(), "reset launch");
}

static long flat_blocks(long n) {
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  return blocks < 1 ? 1 : blocks;
}

// clears the entry word flag[1] (and the attempt's word and counters)
int entry_clear(mhd25_ctx* c) {
  hipLaunchKernelGGL(k_reset_attempt, dim3(1), dim3(64), 0, c->stream, c->d_flag, c->d_counts, 1);
  return check(c, hipGetLastError(), "entry clear launch");
}

// entry snapshot of U (and of the magnetic grids when B is set) into snapU / saveB with the
// admissibility test; clears and then sets the entry word flag[1]
int entry_snapshot(mhd25_ctx* c, const double* U, double* snapU, const double* const* B, double* saveB) {
  const long KN = c->mp.K * c->nn;
  if (c->rec) {
    rt_record(c, RT_RESET, 0, 1, reset_args{c->d_flag, c->d_counts, 1});
    rt_record(c, RT_SNAP_U, 0, flat_blocks(KN), snap_args{U, snapU, KN, c->mp.gamma, c->d_flag});
    if (B)
      for (int k = 0; k < 3; ++k)
        rt_record(c, RT_COPY_CHECK, 0, flat_blocks(c->G), copy_args{B[k], saveB + k * c->G, c->G, c->d_flag});
    return 0;
  }
  hipLaunchKernelGGL(k_reset_attempt, dim3(1), dim3(64), 0, c->stream, c->d_flag, c->d_counts, 1);
  hipLaunchKernelGGL(k_snap_check_U, dim3(flat_blocks(KN)), dim3(256), 0, c->stream, U, snapU, KN, c->mp.gamma,
                     c->d_flag);
  if (B)
    for (int k = 0; k < 3; ++k)
      hipLaunchKernelGGL(k_copy_check, dim3(flat_blocks(c->G)), dim3(256), 0, c->stream, B[k], saveB + k * c->G, c->G,
                         c->d_flag);
  return check(c, hipGetLastError(), "entry snapshot launch");
}

int hydro_face_map(mhd25_ctx* c, int32_t* nbr, int32_t* fmap) {
  const long blocks = (4 * c->mp.K + 255) / 256;
#define FM(P) hipLaunchKernelGGL((k_face_map<P>), dim3(blocks), dim3(256), 0, c->stream, nbr, fmap, c->mp)
  DISPATCH_P(c->p, FM);
#undef FM
  return check(c, hipGetLastError(), "face map launch");
}

int dcopy(mhd25_ctx* c, const double* a, double* b, long n) {
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (c->rec) { rt_record(c, RT_COPY, 0, blocks, copy_args{a, b, n, nullptr}); return 0; }
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, c->stream, a, b, n);
  return check(c, hipGetLastError(), "copy launch");
}

// ---------------------------------------------------------------------------------------------
// Run-table kernels of the small and flat kernels (argument structs per run) and the dispatcher of
// this file's run-table launches.
// ---------------------------------------------------------------------------------------------
__global__ void k_reset_rt(const reset_args* __restrict__ A, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const reset_args& a = A[r];
  if (a.clear_input) gl(a.flag)[1] = 0;
  gl(a.flag)[0] = gl(a.flag)[1];
  gl(a.counts)[0] = 0; gl(a.counts)[1] = 0; gl(a.counts)[2] = 0;
}

// flat kernels: run r owns blocks boff[r] .. boff[r+1) and strides over its n entries with them
__global__ __launch_bounds__(256) void k_copy_rt(const copy_args* __restrict__ A, const int* __restrict__ boff, int nr) {
  const int r = rt_run(boff, nr);
  const copy_args& a = A[r];
  const long stride = (long)(boff[r + 1] - boff[r]) * blockDim.x;
  for (long k = (long)(blockIdx.x - boff[r]) * blockDim.x + threadIdx.x; k < a.n; k += stride) {
    const double v = gl(a.a)[k];
    gl(a.b)[k] = v;
    if (gl(a.flag) && !(fabs(v) <= DBL_MAX)) atomicOr(gl(a.flag) + 1, 2);
  }
}

__global__ __launch_bounds__(256) void k_snap_check_U_rt(const snap_args* __restrict__ A, const int* __restrict__ boff,
                                                         int nr) {
  const int r = rt_run(boff, nr);
  const snap_args& a = A[r];
  const long stride = (long)(boff[r + 1] - boff[r]) * blockDim.x;
  for (long n = (long)(blockIdx.x - boff[r]) * blockDim.x + threadIdx.x; n < a.KN; n += stride)
    snap_check_node(gl(a.U), gl(a.snap), a.KN, a.g, gl(a.flag), n);
}

int hydro_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s) {
  const dim3 g((unsigned)nblocks);
  switch (h.kind) {
    case RT_HYDRO_STAGE: {
      const int P = h.key / 1000, bs = h.key % 1000;
      const hydro_stage_args* A = (const hydro_stage_args*)dargs;
#define RS(P_)                                                                                                       \
  if (bs == 128) hipLaunchKernelGGL((k_hydro_stage_rt<P_, 1, 128>), g, dim3(128), 0, s, A, dboff, nr);              \
  else hipLaunchKernelGGL((k_hydro_stage_rt<P_, 1, 256>), g, dim3(256), 0, s, A, dboff, nr)
      DISPATCH_P(P, RS);
#undef RS
      break;
    }
    case RT_OE_PP: {
      const hydro_oe_pp_args* A = (const hydro_oe_pp_args*)dargs;
#define RO(P_) hipLaunchKernelGGL((k_hydro_oe_pp_rt<P_, MHD_OE_BS>), g, dim3(MHD_OE_BS), 0, s, A, dboff, nr)
      DISPATCH_P(h.key, RO);
#undef RO
      break;
    }
    case RT_LINE_REDUCE: {
      const line_reduce_args* A = (const line_reduce_args*)dargs;
#define RL(NC) hipLaunchKernelGGL((k_line_reduce_rt<NC>), g, dim3(256), 0, s, A, dboff, nr)
      switch (h.key) { case 1: RL(1); break; case 2: RL(2); break; case 3: RL(3); break; case 4: RL(4); break;
                       case 5: RL(5); break; default: return -2; }
#undef RL
      break;
    }
    case RT_GLOBAL_REDUCE: {
      const global_reduce_args* A = (const global_reduce_args*)dargs;
#define RG(NC) hipLaunchKernelGGL((k_global_reduce_rt<NC>), g, dim3(256), 0, s, A, dboff, nr)
      switch (h.key) { case 1: RG(1); break; case 2: RG(2); break; case 3: RG(3); break; case 4: RG(4); break;
                       case 5: RG(5); break; default: return -2; }
#undef RG
      break;
    }
    case RT_RESET:
      hipLaunchKernelGGL(k_reset_rt, dim3((nr + 63) / 64), dim3(64), 0, s, (const reset_args*)dargs, nr);
      break;
    case RT_COPY:
    case RT_COPY_CHECK:
      hipLaunchKernelGGL(k_copy_rt, g, dim3(256), 0, s, (const copy_args*)dargs, dboff, nr);
      break;
    case RT_SNAP_U:
      hipLaunchKernelGGL(k_snap_check_U_rt, g, dim3(256), 0, s, (const snap_args*)dargs, dboff, nr);
      break;
    default:
      return 1;  // not a kind of this file
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
