// Small auxiliary kernels: max reduction, positivity-CFL wave speed and diagnostics.
#include <cfloat>

#include "common.h"

namespace {

__device__ __forceinline__ long wr(long a, long n) { return a >= n ? a - n : a; }
__device__ __forceinline__ long gix2(const MeshP& mp, int B, long ex, long ey, int i, int j) {
  const long NX = (long)mp.nx * B, NY = (long)mp.ny * B;
  return wr(ey * B + j, NY) * NX + wr(ex * B + i, NX);
}

// mode 0: max over n values; mode 1: per column sums of [n][6] for cols 0..3, min for 4..5
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ a, long n, int mode, double* __restrict__ out) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  const int ncol = mode == 0 ? 1 : 6;
  double v[6];
  for (int c = 0; c < ncol; ++c) v[c] = (mode == 0) ? -DBL_MAX : (c < 4 ? 0.0 : DBL_MAX);
  for (long k = t; k < n; k += 256) {
    if (mode == 0) v[0] = fmax(v[0], a[k]);
    else
      for (int c = 0; c < 6; ++c) v[c] = c < 4 ? v[c] + a[k * 6 + c] : fmin(v[c], a[k * 6 + c]);
  }
  for (int c = 0; c < ncol; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < ncol; ++c)
        red[c][t] = mode == 0 ? fmax(red[c][t], red[c][t + w])
                              : (c < 4 ? red[c][t] + red[c][t + w] : fmin(red[c][t], red[c][t + w]));
    __syncthreads();
  }
  if (t < ncol) out[t] = red[t][0];
}

// first level: each block reduces a contiguous chunk of the input into one partial
__global__ __launch_bounds__(256) void k_reduce_partial(const double* __restrict__ a, long n, int mode, long chunk,
                                                        double* __restrict__ part) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  const int ncol = mode == 0 ? 1 : 6;
  const long lo = (long)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double v[6];
  for (int c = 0; c < ncol; ++c) v[c] = (mode == 0) ? -DBL_MAX : (c < 4 ? 0.0 : DBL_MAX);
  for (long k = lo + t; k < hi; k += 256) {
    if (mode == 0) v[0] = fmax(v[0], a[k]);
    else
      for (int c = 0; c < 6; ++c) v[c] = c < 4 ? v[c] + a[k * 6 + c] : fmin(v[c], a[k * 6 + c]);
  }
  for (int c = 0; c < ncol; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < ncol; ++c)
        red[c][t] = mode == 0 ? fmax(red[c][t], red[c][t + w])
                              : (c < 4 ? red[c][t] + red[c][t + w] : fmin(red[c][t], red[c][t + w]));
    __syncthreads();
  }
  if (t < ncol) part[(long)blockIdx.x * ncol + t] = red[t][0];
}

// Largest positivity-CFL wave-speed sum of each element: one thread per GLL_p node, EB elements
// per 256-thread block; the element's B coefficients are staged in LDS and interpolated to the
// node by sum factorisation; the element maximum is taken in LDS (a NaN propagates).
template <int P, int M>
__global__ __launch_bounds__(256) void k_cfl(const double* __restrict__ U, const double* __restrict__ Bx,
                                             const double* __restrict__ By, const double* __restrict__ Bz,
                                             double* __restrict__ out, const MagTab* __restrict__ T, MeshP mp) {
  constexpr int NP = P + 1, NN = NP * NP, EB = 256 / NN, A = M + 2, B = M + 1, AB = A * B, BB = B * B;
  __shared__ double sbx[EB][AB], sby[EB][AB], sbz[EB][BB], ss[EB][NN];
  __shared__ double tWP[NP][A], tGP[NP][B], tVP[NP][B];
  const int tid = threadIdx.x, el = tid / NN, q = tid - el * NN, qi = q % NP, qj = q / NP;
  const long e = (long)blockIdx.x * EB + el;
  const bool act = el < EB && e < mp.K;
  long ex, ey;
  elem_xy(mp, act ? e : 0, ex, ey);
  const long KN = mp.K * NN;
  for (int t = tid; t < NP * A; t += 256) tWP[t / A][t % A] = T->I_W_P[t / A][t % A];
  for (int t = tid; t < NP * B; t += 256) {
    tGP[t / B][t % B] = T->I_G_P[t / B][t % B];
    tVP[t / B][t % B] = T->I_V_P[t / B][t % B];
  }
  if (act) {
    for (int k = q; k < AB; k += NN) {
      sbx[el][k] = Bx[gix2(mp, B, ex, ey, k % A, k / A)];
      sby[el][k] = By[gix2(mp, B, ex, ey, k % B, k / B)];
    }
    for (int k = q; k < BB; k += NN) sbz[el][k] = Bz[gix2(mp, B, ex, ey, k % B, k / B)];
  }
  __syncthreads();
  if (act) {
    const long n = e * NN + q;
    const double r = U[n], ir = 1.0 / r;
    const double ux = U[KN + n] * ir, uy = U[2 * KN + n] * ir, uz = U[3 * KN + n] * ir;
    const double p = (mp.gamma - 1.0) * (U[4 * KN + n] - 0.5 * r * (ux * ux + uy * uy + uz * uz));
    double bx = 0.0, by = 0.0, bz = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < A; ++i) t += tWP[qi][i] * sbx[el][j * A + i];
      bx += tGP[qj][j] * t;
    }
#pragma unroll
    for (int j = 0; j < A; ++j) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) t += tGP[qi][i] * sby[el][j * B + i];
      by += tWP[qj][j] * t;
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i) t += tVP[qi][i] * sbz[el][j * B + i];
      bz += tVP[qj][j] * t;
    }
    const double cf = sqrt((mp.gamma * p + bx * bx + by * by + bz * bz) * ir);
    ss[el][q] = (2.0 * P + 1.0) * ((fabs(ux) + cf) / mp.hx + (fabs(uy) + cf) / mp.hy);
  }
  __syncthreads();
  if (act && q == 0) {
    double mx = 0.0;
    for (int k = 0; k < NN; ++k) {
      const double s = ss[el][k];
      mx = (s > mx || s != s) ? s : mx;
    }
    out[e] = mx;
  }
}

template <int P, int M>
__global__ __launch_bounds__(128) void k_diag(const double* __restrict__ U, const double* __restrict__ Bx,
                                              const double* __restrict__ By, const double* __restrict__ Bz,
                                              double* __restrict__ out, const MagTab* __restrict__ T, MeshP mp) {
  constexpr int NP = P + 1, NN = NP * NP, A = M + 2, B = M + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp.K) return;
  long ex, ey;
  elem_xy(mp, e, ex, ey);
  const long KN = mp.K * NN;
  double mass = 0.0, Em = 0.0, rmin = DBL_MAX, pmin = DBL_MAX;
  for (int q = 0; q < NN; ++q) {
    const long n = e * NN + q;
    const double w = mp.J * T->wp[q % NP] * T->wp[q / NP];
    const double r = U[n];
    const double p = (mp.gamma - 1.0) * (U[4 * KN + n] - (U[KN + n] * U[KN + n] + U[2 * KN + n] * U[2 * KN + n] +
                                                          U[3 * KN + n] * U[3 * KN + n]) / (2.0 * r));
    mass += w * r; Em += w * U[4 * KN + n];
    rmin = fmin(rmin, r); pmin = fmin(pmin, p);
  }
  double mag = 0.0, div2 = 0.0;
  for (int qy = 0; qy < A; ++qy)
    for (int qx = 0; qx < A; ++qx) {
      double bx = 0.0, by = 0.0, bz = 0.0, dxbx = 0.0, dyby = 0.0;
      for (int j = 0; j < B; ++j)
        for (int i = 0; i < A; ++i) {
          const double v = Bx[gix2(mp, B, ex, ey, i, j)];
          bx += T->I_W_Q[qx][i] * T->I_G_Q[qy][j] * v;
          dxbx += T->D_W_Q[qx][i] * T->I_G_Q[qy][j] * v;
        }
      for (int j = 0; j < A; ++j)
        for (int i = 0; i < B; ++i) {
          const double v = By[gix2(mp, B, ex, ey, i, j)];
          by += T->I_G_Q[qx][i] * T->I_W_Q[qy][j] * v;
          dyby += T->I_G_Q[qx][i] * T->D_W_Q[qy][j] * v;
        }
      for (int j = 0; j < B; ++j)
        for (int i = 0; i < B; ++i) bz += T->I_V_Q[qx][i] * T->I_V_Q[qy][j] * Bz[gix2(mp, B, ex, ey, i, j)];
      const double w = mp.J * T->wq[qx] * T->wq[qy];
      const double dv = (2.0 / mp.hx) * dxbx + (2.0 / mp.hy) * dyby;
      mag += w * 0.5 * (bx * bx + by * by + bz * bz);
      div2 += w * dv * dv;
    }
  double* o = out + e * 6;
  o[0] = mass; o[1] = Em; o[2] = mag; o[3] = div2; o[4] = rmin; o[5] = pmin;
}

// Physical coordinates of the nodes of one node set (space 0: GLL_p element nodes [K][p+1][p+1];
// 1..6: the B_x, B_y, B_z, W, N_x, N_y grids).  Grid node (gy, gx) is local node (gx mod (m+1),
// gy mod (m+1)) of element (gx / (m+1), gy / (m+1)).  One thread per node.
__global__ __launch_bounds__(256) void k_node_coords(int space, double* __restrict__ x, double* __restrict__ y,
                                                     const HydroTab* __restrict__ H, const MagTab* __restrict__ T,
                                                     MeshP mp, int p, int m, double x0, double y0) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (space == 0) {
    const int np = p + 1, nn = np * np;
    if (k >= mp.K * nn) return;
    const long e = k / nn;
    const int q = (int)(k - e * nn), i = q % np, j = q / np;
    long ex, ey;
    elem_xy(mp, e, ex, ey);
    x[k] = x0 + mp.hx * ex + 0.5 * (H->xi[i] + 1.0) * mp.hx;
    y[k] = y0 + mp.hy * ey + 0.5 * (H->xi[j] + 1.0) * mp.hy;
    return;
  }
  const int B = m + 1;
  const long NX = (long)mp.nx * B;
  if (k >= NX * mp.ny * B) return;
  const long gy = k / NX, gx = k - gy * NX, ex = gx / B, ey = gy / B;
  const int i = (int)(gx - ex * B), j = (int)(gy - ey * B);
  const double* sx = space == 2 || space == 5 ? T->xg : (space == 3 ? T->xv : T->xw);
  const double* sy = space == 1 || space == 6 ? T->xg : (space == 3 ? T->xv : T->xw);
  x[k] = x0 + mp.hx * ex + 0.5 * (sx[i] + 1.0) * mp.hx;
  y[k] = y0 + mp.hy * ey + 0.5 * (sy[j] + 1.0) * mp.hy;
}

}  // namespace

#define DISPATCH_PM2(p, m, F)                                                                             \
  if (p == 1 && m == 0) { F(1, 0); } else if (p == 1 && m == 1) { F(1, 1); }                              \
  else if (p == 2 && m == 1) { F(2, 1); } else if (p == 2 && m == 2) { F(2, 2); }                         \
  else if (p == 3 && m == 2) { F(3, 2); } else if (p == 3 && m == 3) { F(3, 3); }                         \
  else if (p == 4 && m == 3) { F(4, 3); } else if (p == 4 && m == 4) { F(4, 4); }                         \
  else if (p == 5 && m == 4) { F(5, 4); } else if (p == 5 && m == 5) { F(5, 5); }                         \
  else if (p == 6 && m == 5) { F(6, 5); } else if (p == 6 && m == 6) { F(6, 6); }                         \
  else return -4;

static int ex_chk(mhd25_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) { c->err = std::string(what) + ": " + hipGetErrorString(e); return -2; }
  return 0;
}

// two-level deterministic reduction (fixed partition): mode 0 max of a[n]; mode 1 column sums / mins of a[n][6]
static void reduce2(mhd25_ctx* c, const double* a, long n, int mode, double* d_out) {
  double* part = c->red + 16 + c->mp.K + 64;
  long nb = (n + 4095) / 4096;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  const long chunk = (n + nb - 1) / nb;
  hipLaunchKernelGGL(k_reduce_partial, dim3(nb), dim3(256), 0, c->stream, a, n, mode, chunk, part);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, c->stream, part, nb, mode, d_out);
}

struct max_args {
  const double* a;
  long n;
  double* out;
};

// run-table maximum: one block per run over its n values (max is exact, so the result equals the
// two-level reduction's)
__global__ __launch_bounds__(256) void k_max_rt(const max_args* __restrict__ A, int nr) {
  __shared__ double red[256];
  const max_args a = A[blockIdx.x];
  const int t = threadIdx.x;
  double v = -DBL_MAX;
  for (long k = t; k < a.n; k += 256) v = fmax(v, a.a[k]);
  red[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) *a.out = red[0];
}

int extra_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s) {
  (void)dboff; (void)nblocks;
  if (h.kind != RT_MAX) return 1;
  hipLaunchKernelGGL(k_max_rt, dim3(nr), dim3(256), 0, s, (const max_args*)dargs, nr);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int extra_max_dev(mhd25_ctx* c, const double* a, long n, double* d_out) {
  if (c->rec) { rt_record(c, RT_MAX, 0, 1, max_args{a, n, d_out}); return 0; }
  reduce2(c, a, n, 0, d_out);
  return ex_chk(c, hipGetLastError(), "reduce");
}

int extra_max(mhd25_ctx* c, const double* a, long n, double* host_out) {
  double* d_out = c->red + 0;
  reduce2(c, a, n, 0, d_out);
  int r = ex_chk(c, hipMemcpyAsync(c->h_pinned, d_out, 8, hipMemcpyDeviceToHost, c->stream), "copy");
  if (r) return r;
  r = ex_chk(c, hipStreamSynchronize(c->stream), "sync");
  *host_out = c->h_pinned[0];
  return r;
}

int extra_cfl(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz, double* host_max) {
  const long eb = 256 / ((c->p + 1) * (c->p + 1));
  const long nb = (c->mp.K + eb - 1) / eb;
  double* buf = c->red + 16;
#define CF(P, M) hipLaunchKernelGGL((k_cfl<P, M>), dim3(nb), dim3(256), 0, c->stream, U, Bx, By, Bz, buf, c->d_mt, c->mp)
  DISPATCH_PM2(c->p, c->m, CF);
#undef CF
  return extra_max(c, buf, c->mp.K, host_max);
}

int extra_diagnostics(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz,
                      double* out6) {
  const long nb = (c->mp.K + 127) / 128;
  double* buf = c->Ust;  // 5*K*nn >= 6*K doubles
#define DG(P, M) hipLaunchKernelGGL((k_diag<P, M>), dim3(nb), dim3(128), 0, c->stream, U, Bx, By, Bz, buf, c->d_mt, c->mp)
  DISPATCH_PM2(c->p, c->m, DG);
#undef DG
  reduce2(c, buf, c->mp.K, 1, c->red);
  int r = ex_chk(c, hipMemcpyAsync(c->h_pinned, c->red, 6 * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  if (r) return r;
  r = ex_chk(c, hipStreamSynchronize(c->stream), "sync");
  for (int k = 0; k < 6; ++k) out6[k] = c->h_pinned[k];
  out6[3] = sqrt(out6[3]);
  return r;
}

int extra_node_coords(mhd25_ctx* c, int space, double* x, double* y) {
  const long n = space == 0 ? c->mp.K * c->nn : c->G;
  const long nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_node_coords, dim3(nb), dim3(256), 0, c->stream, space, x, y, c->d_ht, c->d_mt, c->mp, c->p,
                     c->m, c->mesh.x0, c->mesh.y0);
  return ex_chk(c, hipGetLastError(), "node coordinate launch");
}
