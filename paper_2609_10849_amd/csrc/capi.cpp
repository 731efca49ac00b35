// C ABI of the gfx950 library (declared in include/mhd25.h): context management and the host
// control flow of algorithms "Hydrodynamic Euler substep", "Magnetic-velocity substep" and
// "Strang split MHD step".  All arithmetic runs in the HIP kernels; the host only sequences
// launches and reads one reject flag (4 bytes) plus three counters per hydro attempt.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <climits>
#include <cstdint>
#include <new>

#include "common.h"

// launchers (hydro.hip, magnetic.hip, extra.hip)
int hydro_rhs(mhd25_ctx* c, const double* U, double* dU);
int hydro_stage_a(mhd25_ctx* c, const double* Us, const double* Un, double* Ust, double ca, double cb, double tau);
int hydro_stats_only(mhd25_ctx* c, const double* U, int* flag);
int hydro_stage_b(mhd25_ctx* c, const double* Ust, double* Uout, double tau, const int* flag, double* rho_o,
                  double* e_o, double* u_o);
int reset_attempt(mhd25_ctx* c);
int dcopy(mhd25_ctx* c, const double* a, double* b, long n);
int mag_reconstruct_JE(mhd25_ctx* c, const double* u, const double* Bx, const double* By, const double* Bz,
                       const double* eta, double* JE, bool r2);
int mag_update(mhd25_ctx* c, const MagIO& io, int mode);
int mag_velocity_oe(mhd25_ctx* c, double tau, const double* rho, double* u, double* e, const double* Bx,
                    const double* By, const double* Bz);
int mag_velocity_prep(mhd25_ctx* c, const double* rho);
int mag_velocity_apply(mhd25_ctx* c, double tau, const double* rho, double* u, double* e, const double* Bx,
                       const double* By, const double* Bz, bool stats_ready, double* Uc);
int mag_ar_eta(mhd25_ctx* c, const double* rho, const double* u, const double* Bx, const double* By,
               const double* Bz, double* eta);
int mag_to_primitive(mhd25_ctx* c, const double* U, double* rho, double* e, double* u);
int mag_to_conservative(mhd25_ctx* c, const double* rho, const double* e, const double* u, double* U);
int mag_B_from_potential(mhd25_ctx* c, const double* A, double* Bx, double* By);
int extra_max(mhd25_ctx* c, const double* a, long n, double* host_out);
int extra_cfl(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz, double* host_max);
int extra_diagnostics(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz,
                      double* out6);
int extra_node_coords(mhd25_ctx* c, int space, double* x, double* y);
int entry_snapshot(mhd25_ctx* c, const double* U, double* snapU, const double* const* B, double* saveB);
int mag_check_input(mhd25_ctx* c, const double* rho, const double* e, const double* u, const double* Bx,
                    const double* By, const double* Bz);
int hydro_face_map(mhd25_ctx* c, int32_t* nbr, int32_t* fmap);
int mag_dof_maps(mhd25_ctx* c, int32_t* dof);
int noalloc_setup(mhd25_ctx* c);

// fold the recorded (start, stop) pairs into the per-kernel totals
static hipError_t timing_fold(mhd25_ctx* c) {
  if (c->ev_used == 0) return hipSuccess;
  const hipError_t e = hipEventSynchronize(c->ev_pool[c->ev_used - 1]);
  if (e != hipSuccess) return e;
  for (int k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]);
    const int kid = c->ev_kid[k / 2];
    c->t_launch[kid]++; c->t_ms[kid] += ms;
  }
  c->ev_used = 0;
  return hipSuccess;
}

// next free (start, stop) event pair for a launch of kernel kid; a full pool is folded first
hipEvent_t* timing_slot(mhd25_ctx* c, int kid) {
  if ((size_t)(c->ev_used + 2) > c->ev_pool.size()) {
    (void)timing_fold(c);
    if (c->ev_pool.empty()) {
      c->ev_pool.resize(2048);
      c->ev_kid.assign(1024, 0);
      for (auto& ev : c->ev_pool) hipEventCreate(&ev);
    }
  }
  c->ev_kid[c->ev_used / 2] = kid;
  hipEvent_t* s = &c->ev_pool[c->ev_used];
  c->ev_used += 2;
  return s;
}

static int fail(mhd25_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(c, call)                                                                   \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess) return fail(c, _e == hipErrorOutOfMemory ? -3 : -2,             \
                                      std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define TRY(x)            \
  do {                    \
    int _r = (x);         \
    if (_r) return _r;    \
  } while (0)

extern "C" {

void mhd25_default_options(mhd25_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->s_H = 0.02; o->s_M = 0.02; o->C_s = 5.0; o->C_eta = 0.2;
  o->iface_flux = 0; o->max_halvings = 10;
}

const char* mhd25_last_error(const mhd25_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mhd25_set_options(mhd25_ctx* c, const mhd25_options* opt) {
  if (!c || !opt) return -1;
  if (opt->max_halvings < 0 || opt->max_halvings > 60 || opt->s_H < 0 || opt->s_M < 0 || opt->C_s < 0 ||
      opt->C_eta < 0 || (opt->iface_flux != 0 && opt->iface_flux != 1) ||
      (opt->reduced_2d2v != 0 && opt->reduced_2d2v != 1) || (opt->strang_order != 0 && opt->strang_order != 1))
    return fail(c, -1, "invalid options");
  c->opt = *opt;
  return 0;
}

void mhd25_destroy(mhd25_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->d_ht, c->d_mt, c->Un, c->S1, c->S2, c->Ust, c->stats, c->lines, c->glob, c->d_flag,
                  c->d_counts, c->d_flags, c->rho, c->e, c->u, c->eta, c->Y1, c->Y2, c->JE,
                  c->loads, c->saveU, c->saveB, c->red, c->snapU, c->vjp_scratch, c->psi, c->artr, c->dfac};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  for (auto& ev : c->ev_pool) (void)hipEventDestroy(ev);
  delete c;
}

int mhd25_init(const mhd25_mesh_desc* mesh, const mhd25_options* opt, void* stream, mhd25_ctx** out) {
  if (!mesh || !out) return -1;
  *out = nullptr;
  const mhd25_mesh_desc& d = *mesh;
  if (d.nx < 1 || d.ny < 1 || !(d.x1 > d.x0) || !(d.y1 > d.y0) || !(d.gamma > 1.0)) return -1;
  if (d.p < 1 || d.p > MHD_MAXP) return -4;
  if (d.m != d.p && d.m != d.p - 1) return -4;
  if ((long)d.nx * d.ny * (d.m + 1) > MHD_MAX_ELEMENTS) return -1;
  if ((long)d.nx * d.ny * (d.p + 1) * (d.p + 1) >= MHD_MAX_NODES) return -1;
  if (d.walls < 0 || d.walls > 3 || ((d.walls & 1) && d.nx % 2) || ((d.walls & 2) && d.ny % 2)) return -1;
  mhd25_ctx* c = new (std::nothrow) mhd25_ctx();
  if (!c) return -3;
  c->mesh = d;
  mhd25_default_options(&c->opt);
  if (opt && mhd25_set_options(c, opt)) { mhd25_destroy(c); return -1; }
  c->stream = (hipStream_t)stream;
  c->p = d.p; c->m = d.m; c->np = d.p + 1; c->nn = c->np * c->np; c->M1 = d.m + 1;
  c->mp.nx = d.nx; c->mp.ny = d.ny; c->mp.K = (long)d.nx * d.ny;
  meshp_set_division(c->mp);
  c->mp.hx = (d.x1 - d.x0) / d.nx; c->mp.hy = (d.y1 - d.y0) / d.ny;
  c->mp.J = c->mp.hx * c->mp.hy / 4.0; c->mp.gamma = d.gamma;
  c->mp.rhx = 1.0 / c->mp.hx; c->mp.rhy = 1.0 / c->mp.hy;
  c->mp.gk = 0.5 / (c->mp.gamma - 1.0);
  c->mp.walls = d.walls;
  c->mp.bx = (d.walls & 1) ? d.nx / 2 : d.nx; c->mp.by = (d.walls & 2) ? d.ny / 2 : d.ny;
  c->mp.r4K = 1.0 / (4.0 * (double)c->mp.bx * c->mp.by);
  c->mp.r4nx = 1.0 / (4.0 * c->mp.bx); c->mp.r4ny = 1.0 / (4.0 * c->mp.by);
  c->mp.area = (double)((long)c->mp.bx * c->mp.by) * c->mp.hx * c->mp.hy;
  c->G = (long)d.nx * d.ny * c->M1 * c->M1;
  build_hydro_tables(c->p, &c->h_ht);
  build_mag_tables(c->p, c->m, &c->h_mt);
  {  // reciprocal lumped weights of the gathered nodes (a shared node adds its neighbours' weights)
    const int A = c->m + 2, B = c->m + 1;
    const MagTab& t = c->h_mt;
    for (int j = 0; j < B; ++j)
      for (int i = 0; i < B; ++i) {
        const long double wx = (long double)t.ww[i] + (i == 0 ? t.ww[A - 1] : 0.0L);
        const long double wy = (long double)t.ww[j] + (j == 0 ? t.ww[A - 1] : 0.0L);
        const long double J = c->mp.J;
        c->h_mt.rjw[0][j][i] = (double)(1.0L / (J * wx * wy));               // W: GLL in x and y
        c->h_mt.rjw[1][j][i] = (double)(1.0L / (J * (long double)t.wg[i] * wy));  // N_x: Gauss in x
        c->h_mt.rjw[2][j][i] = (double)(1.0L / (J * wx * (long double)t.wg[j]));  // N_y: Gauss in y
      }
  }
  const long K = c->mp.K, KN = K * c->nn, n5 = 5 * KN, G = c->G;
  const int a = c->m + 2, b = c->m + 1;
  const long ny_ = d.ny, nx_ = d.nx;
  auto alloc = [&](void** p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) return fail(c, e == hipErrorOutOfMemory ? -3 : -2, std::string("hipMalloc: ") + hipGetErrorString(e));
    return 0;
  };
  int r = 0;
  r = r ? r : alloc((void**)&c->d_ht, sizeof(HydroTab));
  r = r ? r : alloc((void**)&c->d_mt, sizeof(MagTab));
  r = r ? r : alloc((void**)&c->Un, n5 * 8);
  r = r ? r : alloc((void**)&c->S1, n5 * 8);
  r = r ? r : alloc((void**)&c->S2, n5 * 8);
  r = r ? r : alloc((void**)&c->Ust, n5 * 8);
  r = r ? r : alloc((void**)&c->stats, K * 15 * 8);
  r = r ? r : alloc((void**)&c->lines, (nx_ + ny_) * 15 * 8);
  r = r ? r : alloc((void**)&c->glob, 64 * 8);
  r = r ? r : alloc((void**)&c->d_flag, 64);
  r = r ? r : alloc((void**)&c->d_counts, 64);
  r = r ? r : alloc((void**)&c->d_flags, K);
  r = r ? r : alloc((void**)&c->rho, KN * 8);
  r = r ? r : alloc((void**)&c->e, KN * 8);
  r = r ? r : alloc((void**)&c->u, 3 * KN * 8);
  r = r ? r : alloc((void**)&c->eta, K * 8);
  const long ny = 4 * KN + 3 * G;
  r = r ? r : alloc((void**)&c->Y1, ny * 8);
  r = r ? r : alloc((void**)&c->Y2, ny * 8);
  r = r ? r : alloc((void**)&c->JE, 6 * G * 8);
  r = r ? r : alloc((void**)&c->loads, K * (2 * a * b + a * a) * 8);
  r = r ? r : alloc((void**)&c->saveU, n5 * 8);
  r = r ? r : alloc((void**)&c->saveB, 3 * G * 8);
  r = r ? r : alloc((void**)&c->snapU, n5 * 8);
  r = r ? r : alloc((void**)&c->red, (K + 1024) * 8 * 8);
  // velocity-OE basis: allocated here so that no allocation happens inside a captured step
  r = r ? r : alloc((void**)&c->psi, (size_t)K * psi_stride(c->nn) * 8);
  r = r ? r : alloc((void**)&c->dfac, (size_t)K * (c->p + 1) * 8);
  r = r ? r : alloc((void**)&c->artr, (size_t)K * (8 * (c->m + 2) + 2) * 8);
  if (!r && hipHostMalloc((void**)&c->h_pinned, 4096) != hipSuccess) r = fail(c, -3, "hipHostMalloc");
  if (r) { mhd25_destroy(c); return r; }
  if ((r = noalloc_setup(c)) != 0) { mhd25_destroy(c); return r; }
  if (hipMemcpy(c->d_ht, &c->h_ht, sizeof(HydroTab), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_mt, &c->h_mt, sizeof(MagTab), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->d_flags, 0, K) != hipSuccess) {
    mhd25_destroy(c);
    return -2;
  }
  *out = c;
  return 0;
}

int mhd25_rhs_hydro(mhd25_ctx* c, const double* U, double* dU) {
  if (!c || !U || !dU) return -1;
  return hydro_rhs(c, U, dU);
}

int mhd25_hydro_stage_map(mhd25_ctx* c, double* U, double tau, uint8_t* flags) {
  if (!c || !U) return -1;
  const long n5 = 5 * c->mp.K * c->nn;
  TRY(dcopy(c, U, c->Ust, n5));
  TRY(hydro_stats_only(c, c->Ust, nullptr));
  TRY(hydro_stage_b(c, c->Ust, U, tau, nullptr, nullptr, nullptr, nullptr));
  if (flags) HIPCHK(c, hipMemcpyAsync(flags, c->d_flags, c->mp.K, hipMemcpyDeviceToDevice, c->stream));
  return 0;
}

// one attempt of the SSP-RK(3,3) hydro substep; returns 1 accepted, 0 rejected, 2 inadmissible
// input (the entry check's word, see entry_snapshot), <0 error
// with_prim: the last stage also writes the primitive copy (c->rho, c->e, c->u) of the new state
static int hydro_attempt(mhd25_ctx* c, double* U, double tau, long long* counts, bool with_prim) {
  // U itself serves as U^n: it is written only by the last stage's map, which every thread
  // does for its own nodes after all reads of U^n, and which is skipped when the attempt is rejected
  TRY(reset_attempt(c));
  TRY(hydro_stage_a(c, U, U, c->Ust, 0.0, 1.0, tau));
  TRY(hydro_stage_b(c, c->Ust, c->S1, tau, c->d_flag, nullptr, nullptr, nullptr));
  TRY(hydro_stage_a(c, c->S1, U, c->Ust, 0.75, 0.25, tau));
  TRY(hydro_stage_b(c, c->Ust, c->S2, tau, c->d_flag, nullptr, nullptr, nullptr));
  TRY(hydro_stage_a(c, c->S2, U, c->Ust, 1.0 / 3.0, 2.0 / 3.0, tau));
  // skipped (U untouched) when rejected
  TRY(hydro_stage_b(c, c->Ust, U, tau, c->d_flag, with_prim ? c->rho : nullptr, with_prim ? c->e : nullptr,
                    with_prim ? c->u : nullptr));
  int* hf = (int*)c->h_pinned;
  unsigned long long* hc = (unsigned long long*)(c->h_pinned + 8);
  HIPCHK(c, hipMemcpyAsync(hf, c->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(hc, c->d_counts, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hf[1]) return 2;
  if (hf[0]) return 0;
  counts[0] += (long long)hc[0]; counts[1] += (long long)hc[1]; counts[2] += (long long)hc[2];
  return 1;
}

// with_prim: every accepted attempt also writes the primitive copy of its result, so after an
// accepted substep it holds the final state (the last accepted attempt writes last)
static int hydro_substep_rec(mhd25_ctx* c, double* U, double tau, int depth, mhd25_report* rep,
                             bool with_prim = false) {
  rep->substeps_attempted++;
  rep->max_depth = std::max(rep->max_depth, depth);
  long long cnt[3] = {0, 0, 0};
  int ok = hydro_attempt(c, U, tau, cnt, with_prim);
  if (ok < 0) return ok;
  if (ok == 2) {
    rep->substeps_attempted--;
    c->err = "inadmissible input: a non-finite value or a non-positive nodal density or pressure";
    return 2;
  }
  if (ok) {
    rep->substeps_accepted++;
    rep->n_rho_limited += cnt[0]; rep->n_p_limited += cnt[1]; rep->n_collapsed += cnt[2];
    return 0;
  }
  if (depth + 1 > c->opt.max_halvings) {
    c->err = "hydro substep not accepted within max_halvings";
    return 1;
  }
  TRY(hydro_substep_rec(c, U, 0.5 * tau, depth + 1, rep, with_prim));
  return hydro_substep_rec(c, U, 0.5 * tau, depth + 1, rep, with_prim);
}

int mhd25_hydro_substep(mhd25_ctx* c, double* U, double tau, mhd25_report* rep) {
  if (!c || !U || !(tau > 0.0)) return -1;
  mhd25_report r;
  std::memset(&r, 0, sizeof(r));
  r.dt = tau;
  const long n5 = 5 * c->mp.K * c->nn;
  TRY(entry_snapshot(c, U, c->saveU, nullptr, nullptr));
  int s = hydro_substep_rec(c, U, tau, 0, &r);
  if (s > 0) TRY(dcopy(c, c->saveU, U, n5));
  r.status = s;
  if (rep) *rep = r;
  if (s >= 0) HIPCHK(c, hipStreamSynchronize(c->stream));
  return s;
}

int mhd25_reconstruct_JE(mhd25_ctx* c, const double* u, const double* Bx, const double* By, const double* Bz,
                         const double* eta, double* JE6) {
  if (!c || !u || !Bx || !By || !Bz || !JE6) return -1;
  return mag_reconstruct_JE(c, u, Bx, By, Bz, eta, JE6, false);  // all six grids are returned
}

int mhd25_rhs_magnetic(mhd25_ctx* c, const double* rho, const double* u, const double* Bx, const double* By,
                       const double* Bz, const double* eta, double* de, double* du, double* dBx, double* dBy,
                       double* dBz) {
  if (!c || !rho || !u || !Bx || !By || !Bz || !de || !du || !dBx || !dBy || !dBz) return -1;
  const long G = c->G;
  TRY(mag_reconstruct_JE(c, u, Bx, By, Bz, eta, c->JE, c->opt.reduced_2d2v != 0));
  MagIO io{};
  io.rho = rho; io.us = u; io.bxs = Bx; io.bys = By; io.bzs = Bz;
  io.jx = c->JE; io.jy = c->JE + G; io.jz = c->JE + 2 * G;
  io.ex = c->JE + 3 * G; io.ey = c->JE + 4 * G; io.ez = c->JE + 5 * G;
  io.eta = eta;
  io.oe = de; io.ou = du; io.obx = dBx; io.oby = dBy; io.obz = dBz;
  return mag_update(c, io, 0);
}

int mhd25_ar_eta(mhd25_ctx* c, const double* rho, const double* u, const double* Bx, const double* By,
                 const double* Bz, double* eta) {
  if (!c || !rho || !u || !Bx || !By || !Bz || !eta) return -1;
  return mag_ar_eta(c, rho, u, Bx, By, Bz, eta);
}

int mhd25_velocity_oe(mhd25_ctx* c, double tau, const double* rho, double* u, double* e, const double* Bx,
                      const double* By, const double* Bz) {
  if (!c || !rho || !u || !e || !Bx || !By || !Bz) return -1;
  return mag_velocity_oe(c, tau, rho, u, e, Bx, By, Bz);
}

}  // extern "C"

// the magnetic substep without the entry check (the Strang step's own state is admissible)
// With Uc (the conserved state whose density row holds rho) the substep ends with the exchange back
// to Uc: formed inside the last velocity-OE projection, or by the exchange kernel without velocity OE.
int step_magnetic_impl(mhd25_ctx* c, const double* rho, double* e, double* u, double* Bx, double* By, double* Bz,
                       double tau, mhd25_report* rep, double* Uc) {
  const long KN = c->mp.K * c->nn, G = c->G;
  const double* eta = nullptr;
  double eta_max = 0.0;
  if (c->opt.ar && c->opt.C_eta > 0.0) {
    TRY(mag_ar_eta(c, rho, u, Bx, By, Bz, c->eta));
    eta = c->eta;
    if (rep) TRY(extra_max(c, c->eta, c->mp.K, &eta_max));
  }
  // Y = [e | u | Bx | By | Bz] for the intermediate stages; Y^n is the input itself (each node or
  // DOF is read and written by the same thread in the last stage, so no copy is needed)
  auto parts = [&](double* Y, double** pe, double** pu, double** px, double** py, double** pz) {
    *pe = Y; *pu = Y + KN; *px = Y + 4 * KN; *py = Y + 4 * KN + G; *pz = Y + 4 * KN + 2 * G;
  };
  if (c->opt.oe_mag) TRY(mag_velocity_prep(c, rho));  // rho is frozen over the substep
  const double cas[3] = {0.0, 0.75, 1.0 / 3.0}, cbs[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int s = 0; s < 3; ++s) {
    double *se, *su, *sx, *sy, *sz;
    if (s == 0) { se = e; su = u; sx = Bx; sy = By; sz = Bz; }
    else parts(s == 1 ? c->Y1 : c->Y2, &se, &su, &sx, &sy, &sz);
    double *oe, *ou, *ox, *oy, *oz;
    if (s < 2) parts(s == 0 ? c->Y1 : c->Y2, &oe, &ou, &ox, &oy, &oz);
    else { oe = e; ou = u; ox = Bx; oy = By; oz = Bz; }
    TRY(mag_reconstruct_JE(c, su, sx, sy, sz, eta, c->JE, c->opt.reduced_2d2v != 0));
    MagIO io{};
    io.rho = rho; io.us = su; io.es = se; io.bxs = sx; io.bys = sy; io.bzs = sz;
    io.un = u; io.en = e; io.bxn = Bx; io.byn = By; io.bzn = Bz;
    io.jx = c->JE; io.jy = c->JE + G; io.jz = c->JE + 2 * G;
    io.ex = c->JE + 3 * G; io.ey = c->JE + 4 * G; io.ez = c->JE + 5 * G;
    io.eta = eta;
    io.oe = oe; io.ou = ou; io.obx = ox; io.oby = oy; io.obz = oz;
    io.ca = cas[s]; io.cb = cbs[s]; io.tau = tau;
    io.ustats = c->opt.oe_mag ? c->stats : nullptr;  // the update also forms the sensor's u statistics
    TRY(mag_update(c, io, 1));
    if (c->opt.oe_mag) TRY(mag_velocity_apply(c, tau, rho, ou, oe, ox, oy, oz, true, s == 2 ? Uc : nullptr));
  }
  if (Uc && !c->opt.oe_mag) TRY(mag_to_conservative(c, rho, e, u, Uc));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->eta_max = eta_max; rep->dt = tau;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return 0;
}

extern "C" {

int mhd25_step_magnetic(mhd25_ctx* c, const double* rho, double* e, double* u, double* Bx, double* By, double* Bz,
                        double tau, mhd25_report* rep) {
  if (!c || !rho || !e || !u || !Bx || !By || !Bz || !(tau > 0.0)) return -1;
  TRY(mag_check_input(c, rho, e, u, Bx, By, Bz));
  int* hf = (int*)c->h_pinned;
  HIPCHK(c, hipMemcpyAsync(hf, c->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (*hf) {
    if (rep) { std::memset(rep, 0, sizeof(*rep)); rep->dt = tau; rep->status = 2; }
    return fail(c, 2, "inadmissible input: a non-finite value or a non-positive nodal density or internal energy");
  }
  return step_magnetic_impl(c, rho, e, u, Bx, By, Bz, tau, rep, nullptr);
}

int mhd25_to_primitive(mhd25_ctx* c, const double* U, double* rho, double* e, double* u) {
  if (!c || !U || !rho || !e || !u) return -1;
  return mag_to_primitive(c, U, rho, e, u);
}

int mhd25_to_conservative(mhd25_ctx* c, const double* rho, const double* e, const double* u, double* U) {
  if (!c || !U || !rho || !e || !u) return -1;
  return mag_to_conservative(c, rho, e, u, U);
}

int mhd25_strang_step(mhd25_ctx* c, double* U, double* Bx, double* By, double* Bz, double dt, mhd25_report* rep) {
  if (!c || !U || !Bx || !By || !Bz || !(dt > 0.0)) return -1;
  const long KN = c->mp.K * c->nn, G = c->G;
  mhd25_report r;
  std::memset(&r, 0, sizeof(r));
  r.dt = dt;
  // entry snapshot for the failure path (state restored on a positive return), with the input's
  // admissibility test (status 2 from the first attempt when it fails)
  const double* Bin[3] = {Bx, By, Bz};
  TRY(entry_snapshot(c, U, c->snapU, Bin, c->saveB));
  auto restore = [&](int s) {
    if (s > 0) {
      dcopy(c, c->snapU, U, 5 * KN);
      dcopy(c, c->saveB, Bx, G); dcopy(c, c->saveB + G, By, G); dcopy(c, c->saveB + 2 * G, Bz, G);
      (void)hipStreamSynchronize(c->stream);
    }
    r.status = s;
    if (rep) *rep = r;
    return s;
  };
  mhd25_report h1, m, h2;
  std::memset(&h1, 0, sizeof(h1)); std::memset(&m, 0, sizeof(m)); std::memset(&h2, 0, sizeof(h2));
  int s = 0;
  if (c->opt.strang_order == 0) {
    s = hydro_substep_rec(c, U, 0.5 * dt, 0, &h1, true);  // also leaves (rho, e, u) of U
    if (s != 0) return restore(s);
    TRY(step_magnetic_impl(c, c->rho, c->e, c->u, Bx, By, Bz, dt, &m, U));
    s = hydro_substep_rec(c, U, 0.5 * dt, 0, &h2);
  } else {
    // magnetic-outer composition (the entry word is read by the hydro attempt in the middle)
    TRY(mag_to_primitive(c, U, c->rho, c->e, c->u));
    TRY(step_magnetic_impl(c, c->rho, c->e, c->u, Bx, By, Bz, 0.5 * dt, &m, U));
    s = hydro_substep_rec(c, U, dt, 0, &h1, true);  // also leaves (rho, e, u) of U
    if (s != 0) return restore(s);
    TRY(step_magnetic_impl(c, c->rho, c->e, c->u, Bx, By, Bz, 0.5 * dt, &m, U));
  }
  r.substeps_attempted = h1.substeps_attempted + h2.substeps_attempted;
  r.substeps_accepted = h1.substeps_accepted + h2.substeps_accepted;
  r.max_depth = std::max(h1.max_depth, h2.max_depth);
  r.n_rho_limited = h1.n_rho_limited + h2.n_rho_limited;
  r.n_p_limited = h1.n_p_limited + h2.n_p_limited;
  r.n_collapsed = h1.n_collapsed + h2.n_collapsed;
  r.eta_max = m.eta_max;
  return restore(s);
}

int mhd25_cfl_dt(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz, double cfl,
                 double* dt) {
  if (!c || !U || !Bx || !By || !Bz || !dt || !(cfl > 0)) return -1;
  double mx = 0.0;
  TRY(extra_cfl(c, U, Bx, By, Bz, &mx));
  if (!(mx > 0.0)) return fail(c, 2, "non-finite or zero wave speed");
  *dt = cfl / mx;
  return 0;
}

int mhd25_B_from_potential(mhd25_ctx* c, const double* A, double* Bx, double* By) {
  if (!c || !A || !Bx || !By) return -1;
  return mag_B_from_potential(c, A, Bx, By);
}

int mhd25_diagnostics(mhd25_ctx* c, const double* U, const double* Bx, const double* By, const double* Bz,
                      double* out6) {
  if (!c || !U || !Bx || !By || !Bz || !out6) return -1;
  return extra_diagnostics(c, U, Bx, By, Bz, out6);
}

int mhd25_node_coords(mhd25_ctx* c, int32_t space, double* x, double* y) {
  if (!c || !x || !y || space < 0 || space > 6) return -1;
  return extra_node_coords(c, space, x, y);
}

int mhd25_get_maps(mhd25_ctx* c, int32_t* elem_nbr, int32_t* dof_maps) {
  if (!c || !elem_nbr) return -1;
  const long A = c->m + 2, B = c->m + 1;
  if (c->mp.K * c->nn > INT32_MAX || c->G > INT32_MAX ||
      c->mp.K * (4 * c->np + 4 * A * B + A * A + B * B) > INT32_MAX)
    return fail(c, -1, "maps exceed the int32 index range");
  TRY(hydro_face_map(c, elem_nbr, dof_maps));
  if (dof_maps) TRY(mag_dof_maps(c, dof_maps + 4 * c->mp.K * c->np));
  return 0;
}

int mhd25_decisions(const mhd25_ctx* c, uint8_t* host_flags, int64_t n) {
  if (!c || !host_flags || n < c->mp.K) return -1;
  mhd25_ctx* cc = const_cast<mhd25_ctx*>(c);
  HIPCHK(cc, hipMemcpyAsync(host_flags, c->d_flags, c->mp.K, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(cc, hipStreamSynchronize(c->stream));
  return 0;
}

int mhd25_timing_enable(mhd25_ctx* c, int32_t on) {
  if (!c) return -1;
  c->timing = on ? 1 : 0;
  return 0;
}

int mhd25_timing_read(mhd25_ctx* c, int32_t kid, int64_t* launches, double* total_ms) {
  if (!c || kid < 0 || kid > 9 || !launches || !total_ms) return -1;
  HIPCHK(c, timing_fold(c));
  *launches = c->t_launch[kid];
  *total_ms = c->t_ms[kid];
  c->t_launch[kid] = 0; c->t_ms[kid] = 0.0;
  return 0;
}

}  // extern "C"
