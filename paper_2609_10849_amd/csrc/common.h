// Internal definitions of the gfx950 library: device tables, mesh parameters, context.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mhd25.h"

#define MHD_MAXP 6
#define MHD_MAXN 8  // max points of any 1D node set used (p+1 <= 7, m+2 <= 8)

// 1D tables of the DGSEM degree p (section "Nodal bases, quadrature, and mass matrices").
struct HydroTab {
  double xi[MHD_MAXN], w[MHD_MAXN];    // GLL_p nodes / weights
  double Shat[MHD_MAXN][MHD_MAXN];     // (Q - Q^T)_{ir} / w_i : skew flux-differencing weights
  double Tf[MHD_MAXN][MHD_MAXN];       // forward discrete Legendre transform Tf[a][i] = w_i P_a(xi_i)/n_a
  double V[MHD_MAXN][MHD_MAXN];        // V[i][a] = P_a(xi_i)
  double Dr0[MHD_MAXN][MHD_MAXN];      // r-th derivative of l_i at -1 (reference coordinate)
  double Drp[MHD_MAXN][MHD_MAXN];      // r-th derivative of l_i at +1
  double fr[MHD_MAXN];                 // OE sensor factor (2r+1) 2^r / (2 r!)
  int ka[MHD_MAXN * MHD_MAXN];         // shell-ordered tensor Legendre basis: k -> (a, b)
  int kb[MHD_MAXN * MHD_MAXN];
  int ksh[MHD_MAXN * MHD_MAXN];        // shell index max(a, b)
};

// 1D interpolation (I) and derivative (D) matrices between the node sets of the magnetic
// complex; names read  <op>_<source>_<target>[target][source].
//   P: GLL_p (p+1)   W: GLL_{m+1} (m+2)   G: Gauss_m (m+1)   V: GLL_m (m+1)   Q: Gauss_{m+1} (m+2)
struct MagTab {
  double xw[MHD_MAXN], ww[MHD_MAXN];   // GLL_{m+1}
  double xg[MHD_MAXN], wg[MHD_MAXN];   // Gauss_m
  double xq[MHD_MAXN], wq[MHD_MAXN];   // Gauss_{m+1}
  double xv[MHD_MAXN], wv[MHD_MAXN];   // GLL_m
  double xp[MHD_MAXN], wp[MHD_MAXN];   // GLL_p
  double I_W_Q[MHD_MAXN][MHD_MAXN], D_W_Q[MHD_MAXN][MHD_MAXN], I_G_Q[MHD_MAXN][MHD_MAXN];
  double D_W_G[MHD_MAXN][MHD_MAXN], I_V_G[MHD_MAXN][MHD_MAXN];
  double I_P_G[MHD_MAXN][MHD_MAXN], I_P_W[MHD_MAXN][MHD_MAXN];
  double I_W_G[MHD_MAXN][MHD_MAXN], I_G_W[MHD_MAXN][MHD_MAXN], I_V_W[MHD_MAXN][MHD_MAXN];
  double I_G_P[MHD_MAXN][MHD_MAXN], I_W_P[MHD_MAXN][MHD_MAXN], I_V_P[MHD_MAXN][MHD_MAXN];
  double D_W_V[MHD_MAXN][MHD_MAXN], I_G_V[MHD_MAXN][MHD_MAXN];
  double I_G_E[2][MHD_MAXN], I_V_E[2][MHD_MAXN];   // basis values at -1 and +1
  double I_V_Q[MHD_MAXN][MHD_MAXN];
  // 1 / (|J_K| w) of a gathered node, per local position [j][i] < m+1 of its owning element: the
  // lumped weight w sums the contributions of every element sharing the node (W, N_x, N_y nodes).
  // Mesh dependent: set by mhd25_init.
  double rjw[3][MHD_MAXN][MHD_MAXN];
};

// velocity-OE basis table per element: nn rows (one per node) of nn values, each row padded to
// an even length so that every row starts 16-byte aligned
inline constexpr long psi_row(int nn) { return ((long)nn + 1) & ~1L; }
inline constexpr long psi_stride(int nn) { return (long)nn * psi_row(nn); }

struct MeshP {
  int nx, ny;
  long K;
  double hx, hy, J, gamma;
  double rhx, rhy;         // 1 / hx, 1 / hy
  double gk;               // 1 / (2 (gamma - 1)), the energy coefficient of the EC flux
  int walls;               // bit 0 / bit 1: mirror walls normal to x / y, mesh doubled (see mhd25_mesh_desc)
  int bx, by;              // elements per row / column of the box the statistics cover (nx, ny or nx/2, ny/2)
  double r4K, r4nx, r4ny;  // 1 / (4 bx by), 1 / (4 bx), 1 / (4 by): element-average sums to means
  double area;             // bx hx by hy, the box's area: integral sums over the box to means
  unsigned nx_mul;  // element row of e: (e * nx_mul) >> nx_sh, see elem_xy
  int nx_sh;
};

// Largest element count times (m + 1) a context accepts: element indices, grid indices divided
// by m + 1 (and the few idle indices past the end that a block may form) stay below 2^31, which
// row_of relies on.
constexpr long MHD_MAX_ELEMENTS = (1L << 31) - (1L << 16);

// Multiplier and shift for dividing element indices n < 2^31 by nx: with s = ceil(log2 nx) and
// m = ceil(2^(31+s) / nx), m * nx lies in [2^(31+s), 2^(31+s) + 2^s], so floor(n / nx) =
// floor(n * m / 2^(31+s)) for every n < 2^31 (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994, Theorem 4.2); m < 2^32 because nx > 2^(s-1).
inline void meshp_set_division(MeshP& mp) {
  int s = 0;
  while ((1L << s) < (long)mp.nx) ++s;
  mp.nx_sh = 31 + s;
  mp.nx_mul = (unsigned)(((1ULL << mp.nx_sh) + (unsigned long long)mp.nx - 1) / (unsigned long long)mp.nx);
}

// floor(n / nx) for 0 <= n < 2^31
__host__ __device__ __forceinline__ long row_of(const MeshP& mp, long n) {
  return (long)(((unsigned long long)(unsigned)n * mp.nx_mul) >> mp.nx_sh);
}

// Element e = ey * nx + ex split into its column ex and row ey (row-major element order).
__host__ __device__ __forceinline__ void elem_xy(const MeshP& mp, long e, long& ex, long& ey) {
  ey = row_of(mp, e);
  ex = e - ey * mp.nx;
}

// Node arrays: one component of a nodal field holds K (p+1)^2 doubles, fewer than 2^29 (mhd25_init
// rejects larger meshes, whose state arrays alone would exceed the device memory), so the byte offset
// of a node fits 32 bits.  A kernel addresses such an array through a buffer resource (its base in
// scalar registers, its byte size as the range) and one 32-bit offset register per node, instead of
// a 64-bit index product and sum per access; an access beyond the range returns 0 and is not made.
constexpr long MHD_MAX_NODES = 1L << 29;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t node_rsrc(const double* base, long n) {
  // word 3: 32-bit data format, the raw-buffer setting of the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)(unsigned)(n * 8), 0x00020000);
}
__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t r, unsigned boff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned boff, double v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, boff, 0, 0);
}

// 32-bit forms of the element split and of the periodic neighbour index (element indices < 2^31)
__device__ __forceinline__ void elem_xy32(const MeshP& mp, int e, int& ex, int& ey) {
  ey = (int)(((unsigned long long)(unsigned)e * mp.nx_mul) >> mp.nx_sh);
  ex = e - ey * mp.nx;
}
__device__ __forceinline__ int wrap32(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// pointers of one magnetic residual / SSP-stage evaluation (magnetic.hip)
struct MagIO {
  const double *rho, *us, *es, *bxs, *bys, *bzs;  // stage input Y_s (es unused for the residual)
  const double *un, *en, *bxn, *byn, *bzn;        // Y^n (SSP combine only)
  const double *jx, *jy, *jz, *ex, *ey, *ez;      // reconstructed J and E grids
  const double* eta;
  double *oe, *ou, *obx, *oby, *obz;              // outputs
  double* ustats;                                 // optional: [K][3][3] statistics of the new u (SSP combine)
  double ca, cb, tau;
};

// Run-table plans (batched ensembles): with ctx->rec set, the launch helpers append one record per
// kernel launch (its kind, template key, block count and the kernel's argument struct for this run)
// instead of launching; a plan zips the records of all runs into run-table launches.
enum RtKind {
  RT_HYDRO_STAGE, RT_OE_PP, RT_LINE_REDUCE, RT_GLOBAL_REDUCE, RT_RESET, RT_COPY, RT_SNAP_U, RT_COPY_CHECK,
  RT_TO_PRIM, RT_TO_CONS, RT_J_LOADS, RT_E_LOADS, RT_GATHER, RT_MAG_UPDATE, RT_VEL_PREP, RT_VEL_SENSOR,
  RT_VEL_PROJ, RT_B_STATS, RT_AR_TRACES, RT_AR_ETA, RT_MAX, RT_BATCH_ZERO, RT_BATCH_FOLD, RT_NKIND
};
struct RtRecord {
  int kind;
  int key;     // template instantiation (kind-specific encoding)
  long blocks;  // blocks this run needs
  std::vector<unsigned char> args;  // the kernel's argument struct for this run
};

struct mhd25_ctx {
  mhd25_mesh_desc mesh;
  mhd25_options opt;
  hipStream_t stream;
  MeshP mp;
  int p, m, np, nn, M1;
  long G;  // magnetic grid size
  HydroTab* d_ht;
  MagTab* d_mt;
  HydroTab h_ht;
  MagTab h_mt;
  // hydro workspace
  double *Un, *S1, *S2, *Ust, *stats, *lines, *glob;
  int* d_flag;
  unsigned long long* d_counts;  // [3] per attempt
  uint8_t* d_flags;
  // magnetic workspace
  double *rho, *e, *u, *eta, *Y1, *Y2, *Ys, *JE, *loads, *bstat;
  double *saveU, *saveB, *snapU;
  double* red;  // scratch for small reductions
  double* vjp_scratch;  // allocated on the first magnetic VJP
  double* psi;          // rho-weighted orthonormal basis values [K][nn][psi_row(nn)] (velocity OE)
  double* dfac;         // velocity-OE damping factors D_l of the current stage [K][p+1]
  double* artr;         // A.R. face traces and wave-speed maxima [K][8(m+2)+2]
  double* h_pinned;
  std::string err;
  // timing
  int timing;
  int hydro_bs;  // threads per block of the hydro stage kernel (128 or 256; tuned)
  std::vector<hipEvent_t> ev_pool;  // pairs (start, stop) of timed launches
  std::vector<int> ev_kid;          // kernel id of each pair (0 hydro stage, 1 stage map)
  int ev_used;
  long long t_launch[16];  // per timed kernel id (see mhd25_timing_read)
  double t_ms[16];
  std::vector<RtRecord>* rec;  // non-null: launch helpers record instead of launching
};

template <class A>
inline void rt_record(mhd25_ctx* c, int kind, int key, long blocks, const A& a) {
  RtRecord r;
  r.kind = kind; r.key = key; r.blocks = blocks;
  r.args.assign(reinterpret_cast<const unsigned char*>(&a), reinterpret_cast<const unsigned char*>(&a) + sizeof(A));
  c->rec->push_back(std::move(r));
}

// host table builders (tables.cpp)
void build_hydro_tables(int p, HydroTab* t);
void build_mag_tables(int p, int m, MagTab* t);
