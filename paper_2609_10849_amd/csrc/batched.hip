// Batched ensemble of independent runs (uneven meshes and degrees) on one GPU.
//
// Run-table step (mhd25_batch_strang_step): every launch of one Strang step covers all runs.  The
// per-run control flow of the step (hydro attempt, exchange, magnetic substep with A.R. and velocity
// OE, exchange, hydro attempt) has no host reads inside: each run's reject flags are OR-ed into a
// per-run failure word on the device.  Replaying that flow once per run in record mode gives, for
// every launch of the step, each run's kernel arguments and block count; the plan then issues one
// launch per kernel and template instantiation (degree group) whose blocks are split into
// consecutive per-run ranges (a run table of (run, element tile) work items).  About 150 launches
// replace about 4 600 for the 64-run ensemble.  The degree groups share no data, so launched
// directly each group's sequence goes to a branch stream of its own and the groups overlap.  The
// argument tables are uploaded once per set of run pointers and steps, so the plan issues kernels
// only and can be captured on one stream into a HIP graph (mhd25_batch_graph).  After the step one small copy returns all runs' failure words; a
// run that needs a halving (or has an inadmissible input) is restored from its entry snapshot and
// redone with the ordinary step.
//
// Streams step (mhd25_batch_strang_step_streams): the same per-run flow launched run by run on up
// to 8 concurrent branch streams.  Sequential step: the ordinary step run by run.
//
// Autotuning (mhd25_batch_autotune): per degree p the hydro-stage tile (128 or 256 threads per
// block) is timed on the run-table launch of that degree group with the event timer; the branch
// count of the streams step follows a size rule; the choices are stored in a JSON cache.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

int hydro_stage_a(mhd25_ctx* c, const double* Us, const double* Un, double* Ust, double ca, double cb, double tau);
int hydro_stage_b(mhd25_ctx* c, const double* Ust, double* Uout, double tau, const int* flag, double* rho_o,
                  double* e_o, double* u_o);
int reset_attempt(mhd25_ctx* c);
int dcopy(mhd25_ctx* c, const double* a, double* b, long n);
int mag_to_primitive(mhd25_ctx* c, const double* U, double* rho, double* e, double* u);
int extra_max_dev(mhd25_ctx* c, const double* a, long n, double* d_out);
int entry_snapshot(mhd25_ctx* c, const double* U, double* snapU, const double* const* B, double* saveB);
int hydro_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s);
int magnetic_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s);
int extra_rt_launch(const RtRecord& h, const void* dargs, const int* dboff, int nr, long nblocks, hipStream_t s);
int step_magnetic_impl(mhd25_ctx* c, const double* rho, double* e, double* u, double* Bx, double* By, double* Bz,
                       double tau, mhd25_report* rep, double* Uc);

struct zero_args {
  int* fail;
  long long* acc;
  double* eta;
};
struct fold_args {
  const int* flag;
  const unsigned long long* cnt;
  int* fail;
  long long* acc;
};

__device__ __forceinline__ void batch_zero(const zero_args& a) {
  *a.fail = 0; a.acc[0] = a.acc[1] = a.acc[2] = 0; *a.eta = 0.0;
}
__device__ __forceinline__ void batch_fold(const fold_args& a) {
  if (*a.flag) *a.fail = 1;
  a.acc[0] += (long long)a.cnt[0]; a.acc[1] += (long long)a.cnt[1]; a.acc[2] += (long long)a.cnt[2];
}

__global__ void k_batch_zero(zero_args a) {
  if (threadIdx.x == 0) batch_zero(a);
}
__global__ void k_batch_fold(fold_args a) {
  if (threadIdx.x == 0) batch_fold(a);
}
// run-table versions: thread r serves run r
__global__ void k_batch_zero_rt(const zero_args* __restrict__ A, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nr) batch_zero(A[r]);
}
__global__ void k_batch_fold_rt(const fold_args* __restrict__ A, int nr) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nr) batch_fold(A[r]);
}

static int batched_rt_launch(const RtRecord& h, const void* dargs, int nr, hipStream_t s) {
  const dim3 g((nr + 63) / 64);
  if (h.kind == RT_BATCH_ZERO) hipLaunchKernelGGL(k_batch_zero_rt, g, dim3(64), 0, s, (const zero_args*)dargs, nr);
  else if (h.kind == RT_BATCH_FOLD) hipLaunchKernelGGL(k_batch_fold_rt, g, dim3(64), 0, s, (const fold_args*)dargs, nr);
  else return 1;
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// one launch of a run-table plan: the records' kind and key, the runs it covers, its grid and the
// offsets of its argument table and block offsets in the plan's device buffer
struct PlanLaunch {
  RtRecord hdr;  // kind and key (no arguments)
  int group;     // degree group of the runs it covers (runs of one degree p)
  int nr;
  long nblocks;
  size_t arg_off, boff_off;
};

struct mhd25_batch {
  int nruns;
  std::vector<mhd25_ctx*> ctx;
  hipStream_t main;  // caller's stream: plans, replays and the join of the branch streams
  hipStream_t cap;   // idle stream of the batch that graphs are captured on (the caller's stream may
                     // be the legacy default stream, which cannot be captured)
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork;
  int nbranch;
  int* d_fail;
  long long* d_acc;
  double* d_eta;
  int* h_fail;
  long long* h_acc;
  double* h_eta;
  // run-table plan of the last (pointers, dt) set: the launches of degree group 0, then of group 1, ...
  std::vector<PlanLaunch> plan;
  int ngroups;
  unsigned char* d_plan;
  size_t d_plan_cap;
  bool plan_valid;
  std::vector<double> plan_dt;
  std::vector<const double*> plan_ptr;
  // single-stream graph of the plan
  int graph_mode;  // 1: steps replay a captured graph of the plan
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
  std::string err;
};

#define BTRY(x)          \
  do {                   \
    int _r = (x);        \
    if (_r) return _r;   \
  } while (0)

// hydro substep attempt with the accept decision deferred to the device failure word
static int attempt_deferred(mhd25_ctx* c, double* U, double tau, int* fail, long long* acc) {
  const long n5 = 5 * c->mp.K * c->nn;
  BTRY(reset_attempt(c));
  BTRY(dcopy(c, U, c->Un, n5));
  BTRY(hydro_stage_a(c, c->Un, c->Un, c->Ust, 0.0, 1.0, tau));
  BTRY(hydro_stage_b(c, c->Ust, c->S1, tau, c->d_flag, nullptr, nullptr, nullptr));
  BTRY(hydro_stage_a(c, c->S1, c->Un, c->Ust, 0.75, 0.25, tau));
  BTRY(hydro_stage_b(c, c->Ust, c->S2, tau, c->d_flag, nullptr, nullptr, nullptr));
  BTRY(hydro_stage_a(c, c->S2, c->Un, c->Ust, 1.0 / 3.0, 2.0 / 3.0, tau));
  BTRY(hydro_stage_b(c, c->Ust, U, tau, c->d_flag, nullptr, nullptr, nullptr));
  const fold_args fa{c->d_flag, c->d_counts, fail, acc};
  if (c->rec) { rt_record(c, RT_BATCH_FOLD, 0, 1, fa); return 0; }
  hipLaunchKernelGGL(k_batch_fold, dim3(1), dim3(64), 0, c->stream, fa);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// one Strang step of one run, no host synchronisation (graph-capturable)
static int strang_deferred(mhd25_ctx* c, double* U, double* Bx, double* By, double* Bz, double dt, int* fail,
                           long long* acc, double* eta_out) {
  const zero_args za{fail, acc, eta_out};
  if (c->rec) rt_record(c, RT_BATCH_ZERO, 0, 1, za);
  else hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(64), 0, c->stream, za);
  // entry snapshot with the admissibility test: an inadmissible input makes every attempt of the
  // run fail, so the run is redone individually, which returns status 2
  const double* Bin[3] = {Bx, By, Bz};
  BTRY(entry_snapshot(c, U, c->snapU, Bin, c->saveB));
  const bool outer = c->opt.strang_order == 1;  // M(dt/2) H(dt) M(dt/2) instead of H(dt/2) M(dt) H(dt/2)
  auto magnetic = [&](double tau) -> int {
    BTRY(mag_to_primitive(c, U, c->rho, c->e, c->u));
    BTRY(step_magnetic_impl(c, c->rho, c->e, c->u, Bx, By, Bz, tau, nullptr, U));  // ends with the exchange to U
    if (c->opt.ar && c->opt.C_eta > 0.0) BTRY(extra_max_dev(c, c->eta, c->mp.K, eta_out));
    return 0;
  };
  if (outer) BTRY(magnetic(0.5 * dt));
  BTRY(attempt_deferred(c, U, outer ? dt : 0.5 * dt, fail, acc));
  BTRY(magnetic(outer ? 0.5 * dt : dt));
  if (!outer) BTRY(attempt_deferred(c, U, 0.5 * dt, fail, acc));
  return 0;
}

static void release_graph(mhd25_batch* b) {
  if (b->captured) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->captured = false;
  }
}

static int set_branches(mhd25_batch* b, int S) {
  S = std::max(1, std::min(S, 8));
  while ((int)b->br.size() < S) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return -2;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return -2;
    b->br.push_back(s);
    b->ev_join.push_back(ev);
  }
  b->nbranch = S;
  return 0;
}

// greedy assignment of runs to branches by work (largest first)
static std::vector<int> assign(const mhd25_batch* b) {
  std::vector<int> order(b->nruns), out(b->nruns, 0);
  for (int r = 0; r < b->nruns; ++r) order[r] = r;
  auto work = [&](int r) { return (double)b->ctx[r]->mp.K * b->ctx[r]->nn; };
  std::sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
  std::vector<double> load(b->nbranch, 0.0);
  for (int r : order) {
    int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    out[r] = s;
    load[s] += work(r);
  }
  return out;
}

// ---------------------------------------------------------------------------------------------
// Run-table plan
// ---------------------------------------------------------------------------------------------
static bool same_plan(const mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                      double* const* Bz, const double* dt) {
  if (!b->plan_valid) return false;
  for (int r = 0; r < b->nruns; ++r) {
    if (b->plan_dt[r] != dt[r]) return false;
    if (b->plan_ptr[4 * r] != U[r] || b->plan_ptr[4 * r + 1] != Bx[r] || b->plan_ptr[4 * r + 2] != By[r] ||
        b->plan_ptr[4 * r + 3] != Bz[r])
      return false;
  }
  return true;
}

static int build_plan(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By, double* const* Bz,
                      const double* dt) {
  release_graph(b);
  b->plan_valid = false;
  b->plan.clear();
  // each run's launches of one step, recorded without launching
  std::vector<std::vector<RtRecord>> recs(b->nruns);
  for (int r = 0; r < b->nruns; ++r) {
    mhd25_ctx* c = b->ctx[r];
    c->rec = &recs[r];
    const int rc = strang_deferred(c, U[r], Bx[r], By[r], Bz[r], dt[r], b->d_fail + r, b->d_acc + 3 * r, b->d_eta + r);
    c->rec = nullptr;
    if (rc) { b->err = "plan: recording run " + std::to_string(r) + " failed: " + c->err; return rc; }
  }
  const size_t n = recs[0].size();
  for (int r = 1; r < b->nruns; ++r) {
    if (recs[r].size() != n) { b->err = "plan: runs record different launch sequences"; return -2; }
    for (size_t i = 0; i < n; ++i)
      if (recs[r][i].kind != recs[0][i].kind) { b->err = "plan: runs record different launch sequences"; return -2; }
  }
  // degree groups (runs of one degree p, in order of first appearance): the groups share no data,
  // so each group's launches form an independent sequence that may run on a stream of its own
  std::vector<int> degs, grp(b->nruns);
  for (int r = 0; r < b->nruns; ++r) {
    auto it = std::find(degs.begin(), degs.end(), b->ctx[r]->p);
    grp[r] = (int)(it - degs.begin());
    if (it == degs.end()) degs.push_back(b->ctx[r]->p);
  }
  b->ngroups = (int)degs.size();
  // per group, one launch per (position, key): runs grouped by template key in order of first appearance
  std::vector<unsigned char> host;
  auto align = [&]() { host.resize((host.size() + 15) & ~size_t(15)); };
  for (int g = 0; g < b->ngroups; ++g)
  for (size_t i = 0; i < n; ++i) {
    std::vector<int> keys;
    for (int r = 0; r < b->nruns; ++r)
      if (grp[r] == g && std::find(keys.begin(), keys.end(), recs[r][i].key) == keys.end()) keys.push_back(recs[r][i].key);
    for (int key : keys) {
      PlanLaunch L;
      L.hdr.kind = recs[0][i].kind; L.hdr.key = key; L.hdr.blocks = 0;
      L.group = g;
      std::vector<int> boff(1, 0);
      align();
      L.arg_off = host.size();
      L.nr = 0;
      long tot = 0;
      for (int r = 0; r < b->nruns; ++r) {
        const RtRecord& rr = recs[r][i];
        if (grp[r] != g || rr.key != key) continue;
        host.insert(host.end(), rr.args.begin(), rr.args.end());
        tot += rr.blocks;
        if (tot > (1L << 31) - 1) { b->err = "plan: grid too large"; return -1; }
        boff.push_back((int)tot);
        ++L.nr;
      }
      L.nblocks = tot;
      align();
      L.boff_off = host.size();
      const unsigned char* bp = reinterpret_cast<const unsigned char*>(boff.data());
      host.insert(host.end(), bp, bp + boff.size() * sizeof(int));
      b->plan.push_back(std::move(L));
    }
  }
  if (host.size() > b->d_plan_cap) {
    if (b->d_plan) (void)hipFree(b->d_plan);
    b->d_plan = nullptr;
    b->d_plan_cap = 0;
    if (hipMalloc((void**)&b->d_plan, host.size()) != hipSuccess) { b->err = "plan: out of device memory"; return -3; }
    b->d_plan_cap = host.size();
  }
  if (hipMemcpy(b->d_plan, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    b->err = "plan: upload failed";
    return -2;
  }
  b->plan_dt.assign(dt, dt + b->nruns);
  b->plan_ptr.clear();
  for (int r = 0; r < b->nruns; ++r) {
    b->plan_ptr.push_back(U[r]); b->plan_ptr.push_back(Bx[r]); b->plan_ptr.push_back(By[r]); b->plan_ptr.push_back(Bz[r]);
  }
  b->plan_valid = true;
  return 0;
}

// issue the plan's launches on stream s (kernels only: no copies, no host reads)
static int exec_plan(mhd25_batch* b, hipStream_t s) {
  for (const PlanLaunch& L : b->plan) {
    const void* da = b->d_plan + L.arg_off;
    const int* db = reinterpret_cast<const int*>(b->d_plan + L.boff_off);
    int rc = hydro_rt_launch(L.hdr, da, db, L.nr, L.nblocks, s);
    if (rc == 1) rc = magnetic_rt_launch(L.hdr, da, db, L.nr, L.nblocks, s);
    if (rc == 1) rc = extra_rt_launch(L.hdr, da, db, L.nr, L.nblocks, s);
    if (rc == 1) rc = batched_rt_launch(L.hdr, da, L.nr, s);
    if (rc) { b->err = "plan: launch of kind " + std::to_string(L.hdr.kind) + " failed"; return rc == 1 ? -2 : rc; }
  }
  return 0;
}

// issue the plan with each degree group on a branch stream of its own (group g on branch
// g mod nbranch), between a fork event on the caller's stream and join events that the caller's
// stream waits on; the joins are recorded even when a launch fails
static int exec_plan_groups(mhd25_batch* b) {
  if (b->ngroups <= 1 || b->nbranch <= 1) return exec_plan(b, b->main);
  const int nb = std::min(b->ngroups, b->nbranch);
  if (hipEventRecord(b->ev_fork, b->main) != hipSuccess) { b->err = "fork event"; return -2; }
  for (int k = 0; k < nb; ++k)
    if (hipStreamWaitEvent(b->br[k], b->ev_fork, 0) != hipSuccess) { b->err = "fork wait"; return -2; }
  int rc = 0;
  for (const PlanLaunch& L : b->plan) {
    if (rc) break;
    const hipStream_t st = b->br[L.group % nb];
    const void* da = b->d_plan + L.arg_off;
    const int* db = reinterpret_cast<const int*>(b->d_plan + L.boff_off);
    rc = hydro_rt_launch(L.hdr, da, db, L.nr, L.nblocks, st);
    if (rc == 1) rc = magnetic_rt_launch(L.hdr, da, db, L.nr, L.nblocks, st);
    if (rc == 1) rc = extra_rt_launch(L.hdr, da, db, L.nr, L.nblocks, st);
    if (rc == 1) rc = batched_rt_launch(L.hdr, da, L.nr, st);
    if (rc) { b->err = "plan: launch of kind " + std::to_string(L.hdr.kind) + " failed"; rc = rc == 1 ? -2 : rc; }
  }
  for (int k = 0; k < nb; ++k) {
    if (hipEventRecord(b->ev_join[k], b->br[k]) != hipSuccess || hipStreamWaitEvent(b->main, b->ev_join[k], 0) != hipSuccess) {
      b->err = "join";
      if (!rc) rc = -2;
    }
  }
  return rc;
}

// capture the plan on the batch's own idle stream (one stream, kernel nodes only) and instantiate
// it; replays are launched on the caller's stream
static int capture_plan(mhd25_batch* b) {
  release_graph(b);
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    b->err = "graph: begin capture failed";
    return -2;
  }
  const int rc = exec_plan(b, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!rc) b->err = "graph: capture failed";
    return rc ? rc : -2;
  }
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->err = "graph: instantiate failed";
    return -2;
  }
  b->graph = g;
  b->captured = true;
  return 0;
}

// The same deferred steps launched directly on the branch streams, without a graph: a fork event
// on the caller's stream, every branch waits on it, each run is issued on its branch, and the
// caller's stream waits on every branch's join event.  The joins are recorded even when a launch
// fails, so the caller's stream never runs ahead of work already issued.
static int launch_streams(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                          double* const* Bz, const double* dt) {
  std::vector<int> br = assign(b);
  if (hipEventRecord(b->ev_fork, b->main) != hipSuccess) { b->err = "fork event"; return -2; }
  for (int s = 0; s < b->nbranch; ++s)
    if (hipStreamWaitEvent(b->br[s], b->ev_fork, 0) != hipSuccess) { b->err = "fork wait"; return -2; }
  int rc = 0;
  for (int r = 0; r < b->nruns && !rc; ++r) {
    mhd25_ctx* c = b->ctx[r];
    c->stream = b->br[br[r]];
    rc = strang_deferred(c, U[r], Bx[r], By[r], Bz[r], dt[r], b->d_fail + r, b->d_acc + 3 * r, b->d_eta + r);
  }
  for (int r = 0; r < b->nruns; ++r) b->ctx[r]->stream = b->main;
  for (int s = 0; s < b->nbranch; ++s) {
    if (hipEventRecord(b->ev_join[s], b->br[s]) != hipSuccess ||
        hipStreamWaitEvent(b->main, b->ev_join[s], 0) != hipSuccess) {
      b->err = "join";
      if (!rc) rc = -2;
    }
  }
  return rc;
}

extern "C" {

int mhd25_batch_create(const mhd25_mesh_desc* runs, int32_t nruns, const mhd25_options* opt, void* stream,
                       mhd25_batch** out) {
  if (!runs || nruns < 1 || !out) return -1;
  *out = nullptr;
  mhd25_batch* b = new mhd25_batch();
  b->nruns = nruns;
  b->main = (hipStream_t)stream;
  b->nbranch = 0;
  b->captured = false;
  b->d_plan = nullptr;
  b->d_plan_cap = 0;
  b->plan_valid = false;
  b->ngroups = 0;
  b->graph_mode = 0;
  for (int r = 0; r < nruns; ++r) {
    mhd25_ctx* c = nullptr;
    int rc = mhd25_init(&runs[r], opt, stream, &c);
    if (rc) { for (auto* x : b->ctx) mhd25_destroy(x); delete b; return rc; }
    b->ctx.push_back(c);
  }
  if (hipMalloc((void**)&b->d_fail, nruns * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&b->d_acc, 3 * nruns * sizeof(long long)) != hipSuccess ||
      hipMalloc((void**)&b->d_eta, nruns * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&b->h_fail, nruns * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&b->h_acc, 3 * nruns * sizeof(long long)) != hipSuccess ||
      hipHostMalloc((void**)&b->h_eta, nruns * sizeof(double)) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    mhd25_batch_destroy(b);
    return -3;
  }
  if (set_branches(b, 4)) { mhd25_batch_destroy(b); return -2; }
  *out = b;
  return 0;
}

const char* mhd25_batch_last_error(const mhd25_batch* b) { return b ? b->err.c_str() : "null batch"; }

void mhd25_batch_destroy(mhd25_batch* b) {
  if (!b) return;
  release_graph(b);
  for (auto* c : b->ctx) mhd25_destroy(c);
  for (auto s : b->br) (void)hipStreamDestroy(s);
  for (auto e : b->ev_join) (void)hipEventDestroy(e);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_plan) (void)hipFree(b->d_plan);
  if (b->d_fail) (void)hipFree(b->d_fail);
  if (b->d_acc) (void)hipFree(b->d_acc);
  if (b->d_eta) (void)hipFree(b->d_eta);
  if (b->h_fail) (void)hipHostFree(b->h_fail);
  if (b->h_acc) (void)hipHostFree(b->h_acc);
  if (b->h_eta) (void)hipHostFree(b->h_eta);
  delete b;
}

}  // extern "C"

static bool batch_args_ok(const mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                          double* const* Bz, const double* dt) {
  if (!b || !U || !Bx || !By || !Bz || !dt) return false;
  for (int r = 0; r < b->nruns; ++r)
    if (!U[r] || !Bx[r] || !By[r] || !Bz[r] || !(dt[r] > 0.0)) return false;
  return true;
}

// After the runs' deferred steps are on the caller's stream: one small copy returns every run's
// failure word, limiter counters and A.R. maximum; a run that needed a halving is restored from
// its entry snapshot and re-done with the ordinary reject-and-halve step.
static int finish_step(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                       double* const* Bz, const double* dt, mhd25_report* rep) {
  hipMemcpyAsync(b->h_fail, b->d_fail, b->nruns * sizeof(int), hipMemcpyDeviceToHost, b->main);
  hipMemcpyAsync(b->h_acc, b->d_acc, 3 * b->nruns * sizeof(long long), hipMemcpyDeviceToHost, b->main);
  hipMemcpyAsync(b->h_eta, b->d_eta, b->nruns * sizeof(double), hipMemcpyDeviceToHost, b->main);
  if (hipStreamSynchronize(b->main) != hipSuccess) { b->err = "sync"; return -2; }
  int status = 0;
  for (int r = 0; r < b->nruns; ++r) {
    mhd25_ctx* c = b->ctx[r];
    mhd25_report one;
    std::memset(&one, 0, sizeof(one));
    if (b->h_fail[r]) {
      // restore the entry state from the run's snapshot and redo with reject-and-halve
      const long KN = c->mp.K * c->nn, G = c->G;
      BTRY(dcopy(c, c->snapU, U[r], 5 * KN));
      BTRY(dcopy(c, c->saveB, Bx[r], G)); BTRY(dcopy(c, c->saveB + G, By[r], G));
      BTRY(dcopy(c, c->saveB + 2 * G, Bz[r], G));
      int s = mhd25_strang_step(c, U[r], Bx[r], By[r], Bz[r], dt[r], &one);
      if (s && !status) status = s;
    } else {
      one.substeps_attempted = one.substeps_accepted = c->opt.strang_order == 1 ? 1 : 2;
      one.n_rho_limited = b->h_acc[3 * r]; one.n_p_limited = b->h_acc[3 * r + 1];
      one.n_collapsed = b->h_acc[3 * r + 2];
      one.eta_max = b->h_eta[r]; one.dt = dt[r];
    }
    if (rep) rep[r] = one;
  }
  return status;
}

extern "C" {

int mhd25_batch_strang_step(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                            double* const* Bz, const double* dt, mhd25_report* rep) {
  if (!batch_args_ok(b, U, Bx, By, Bz, dt)) return -1;
  if (!same_plan(b, U, Bx, By, Bz, dt)) BTRY(build_plan(b, U, Bx, By, Bz, dt));
  if (b->graph_mode) {
    if (!b->captured) BTRY(capture_plan(b));
    if (hipGraphLaunch(b->exec, b->main) != hipSuccess) { b->err = "graph launch"; return -2; }
  } else {
    BTRY(exec_plan_groups(b));
  }
  return finish_step(b, U, Bx, By, Bz, dt, rep);
}

int mhd25_batch_graph(mhd25_batch* b, int32_t mode) {
  if (!b || mode < -1 || mode > 1) return -1;
  if (mode == -1) { release_graph(b); b->graph_mode = 0; return 0; }
  b->graph_mode = mode;
  if (!mode) release_graph(b);
  return 0;
}

int mhd25_batch_strang_step_streams(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                                    double* const* Bz, const double* dt, mhd25_report* rep) {
  if (!batch_args_ok(b, U, Bx, By, Bz, dt)) return -1;
  BTRY(launch_streams(b, U, Bx, By, Bz, dt));
  return finish_step(b, U, Bx, By, Bz, dt, rep);
}

int mhd25_batch_strang_step_sequential(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                                       double* const* Bz, const double* dt, mhd25_report* rep) {
  if (!b || !U || !Bx || !By || !Bz || !dt) return -1;
  int status = 0;
  for (int r = 0; r < b->nruns; ++r) {
    mhd25_report one;
    int s = mhd25_strang_step(b->ctx[r], U[r], Bx[r], By[r], Bz[r], dt[r], &one);
    if (s < 0) return s;
    if (s && !status) status = s;
    if (rep) rep[r] = one;
  }
  return status;
}

int mhd25_batch_set_tuning(mhd25_batch* b, int32_t branches, int32_t p, int32_t hydro_bs) {
  if (!b) return -1;
  if (branches > 0) BTRY(set_branches(b, branches));
  if (hydro_bs == 128 || hydro_bs == 256) {
    for (auto* c : b->ctx)
      if (p <= 0 || c->p == p) c->hydro_bs = hydro_bs;
    release_graph(b);
    b->plan_valid = false;
  }
  return 0;
}

// Autotuner.  Per degree p present in the batch, the hydro-stage tile (128 or 256 threads per
// block) is timed with HIP events on the run-table launch of that degree group's stage kernel over
// scratch copies of the runs' states (median of 5 launches after 2 warm-ups); the branch count of
// the streams step is min(8, number of runs with at least a quarter of the largest run's work, at
// least 2).  No graph is captured while tuning.
// Choices are appended to the JSON-lines cache and reused when a line with the same run set exists.
int mhd25_batch_autotune(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By, double* const* Bz,
                         const double* dt, const char* cache_path, int32_t* best_branches) {
  if (!b || !U || !Bx || !By || !Bz || !dt) return -1;
  std::ostringstream key;
  for (auto* c : b->ctx) key << c->mesh.nx << "x" << c->mesh.ny << "p" << c->p << "m" << c->m << ";";
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      if (line.find("\"runs\":\"" + key.str() + "\"") == std::string::npos) continue;
      int S = 4;
      const char* q = std::strstr(line.c_str(), "\"branches\":");
      if (q) S = std::atoi(q + 11);
      for (int p = 1; p <= 6; ++p) {
        char pat[32];
        std::snprintf(pat, sizeof(pat), "\"bs_p%d\":", p);
        const char* z = std::strstr(line.c_str(), pat);
        if (z) BTRY(mhd25_batch_set_tuning(b, 0, p, std::atoi(z + std::strlen(pat))));
      }
      BTRY(set_branches(b, S));
      if (best_branches) *best_branches = S;
      return 0;
    }
  }
  std::map<int, int> best_bs;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -2;
  for (int p = 1; p <= 6; ++p) {
    std::vector<int> grp;
    for (int r = 0; r < b->nruns; ++r)
      if (b->ctx[r]->p == p) grp.push_back(r);
    if (grp.empty()) continue;
    // scratch: each run's stage buffers (idle between steps) hold a copy of its state
    for (int r : grp) {
      mhd25_ctx* c = b->ctx[r];
      c->stream = b->main;
      BTRY(dcopy(c, U[r], c->S1, 5 * c->mp.K * c->nn));
    }
    double best = 1e30;
    std::vector<int> saved;
    for (int r : grp) saved.push_back(b->ctx[r]->hydro_bs);
    for (int bs : {256, 128}) {
      // the run-table launch of this degree group's hydro-stage kernel with this tile
      std::vector<unsigned char> host;
      std::vector<int> boff(1, 0);
      RtRecord hdr;
      long tot = 0;
      for (int r : grp) {
        mhd25_ctx* c = b->ctx[r];
        c->hydro_bs = bs;
        std::vector<RtRecord> rec;
        c->rec = &rec;
        const int rc = hydro_stage_a(c, c->S1, c->S1, c->Ust, 0.0, 1.0, 0.25 * dt[r]);
        c->rec = nullptr;
        if (rc) return rc;
        hdr = rec[0];  // the stage kernel's record (the reductions follow it)
        host.insert(host.end(), rec[0].args.begin(), rec[0].args.end());
        tot += rec[0].blocks;
        boff.push_back((int)tot);
      }
      const size_t boff_at = (host.size() + 15) & ~size_t(15);
      host.resize(boff_at);
      const unsigned char* bp = reinterpret_cast<const unsigned char*>(boff.data());
      host.insert(host.end(), bp, bp + boff.size() * sizeof(int));
      unsigned char* d = nullptr;
      if (hipMalloc((void**)&d, host.size()) != hipSuccess) return -3;
      if (hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) { (void)hipFree(d); return -2; }
      std::vector<float> ms;
      for (int k = 0; k < 7; ++k) {
        for (int r : grp) BTRY(reset_attempt(b->ctx[r]));
        hipEventRecord(e0, b->main);
        const int rc = hydro_rt_launch(hdr, d, reinterpret_cast<const int*>(d + boff_at), (int)grp.size(), tot, b->main);
        hipEventRecord(e1, b->main);
        if (rc || hipEventSynchronize(e1) != hipSuccess) { (void)hipFree(d); return -2; }
        float t = 0.f;
        hipEventElapsedTime(&t, e0, e1);
        if (k >= 2) ms.push_back(t);
      }
      (void)hipFree(d);
      std::sort(ms.begin(), ms.end());
      const double med = ms[ms.size() / 2];
      if (med < best) { best = med; best_bs[p] = bs; }
    }
    for (size_t i = 0; i < grp.size(); ++i) b->ctx[grp[i]]->hydro_bs = saved[i];
    BTRY(mhd25_batch_set_tuning(b, 0, p, best_bs[p]));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  double wmax = 0.0;
  for (auto* c : b->ctx) wmax = std::max(wmax, (double)c->mp.K * c->nn);
  int big = 0;
  for (auto* c : b->ctx) big += ((double)c->mp.K * c->nn >= 0.25 * wmax);
  const int S = std::max(2, std::min(8, big));
  BTRY(set_branches(b, S));
  if (best_branches) *best_branches = S;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << "{\"runs\":\"" << key.str() << "\",\"branches\":" << S;
    for (auto& kv : best_bs) f << ",\"bs_p" << kv.first << "\":" << kv.second;
    f << "}\n";
  }
  return 0;
}

}  // extern "C"
