// Batched ensemble of independent runs (uneven meshes and degrees) on one GPU.
//
// One Strang step of every run is captured into a single HIP graph.  The graph forks into S
// branch streams (runs assigned greedily by size), so small runs execute concurrently instead of
// queueing behind each other; inside the graph no host reads happen: each run's hydro reject
// flags are OR-ed into a per-run failure word and its limiter counters accumulated on the device.
// After a replay one small copy returns all runs' words; a run that needs a halving is restored
// from its entry snapshot and re-done on the ordinary (uncaptured) path with reject-and-halve.
// The graph is re-captured when a run's dt or array pointers change.
//
// Autotuning (mhd25_batch_autotune): per degree p the hydro-stage tile (128 or 256 threads per
// block) is timed with plain launches on a scratch copy; the branch count follows a size rule; the
// choices are stored in a JSON cache.
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
int mag_to_conservative(mhd25_ctx* c, const double* rho, const double* e, const double* u, double* U);
int extra_max_dev(mhd25_ctx* c, const double* a, long n, double* d_out);
int entry_snapshot(mhd25_ctx* c, const double* U, double* snapU, const double* const* B, double* saveB);
int step_magnetic_impl(mhd25_ctx* c, const double* rho, double* e, double* u, double* Bx, double* By, double* Bz,
                       double tau, mhd25_report* rep);

__global__ void k_batch_zero(int* fail, long long* acc, double* eta) {
  if (threadIdx.x == 0) { *fail = 0; acc[0] = acc[1] = acc[2] = 0; *eta = 0.0; }
}

__global__ void k_batch_fold(const int* flag, const unsigned long long* cnt, int* fail, long long* acc) {
  if (threadIdx.x == 0) {
    if (*flag) *fail = 1;
    acc[0] += (long long)cnt[0]; acc[1] += (long long)cnt[1]; acc[2] += (long long)cnt[2];
  }
}

struct mhd25_batch {
  int nruns;
  std::vector<mhd25_ctx*> ctx;
  hipStream_t main;   // caller's stream (replays are launched here)
  hipStream_t cap;    // non-blocking stream the graph is captured on
  hipEvent_t ev_cap;  // orders the capture stream after the caller's prior work
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
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
  std::vector<double> cap_dt;
  std::vector<const double*> cap_ptr;
  std::string err;
  bool allow_capture;  // false: the captured step refuses to run (see mhd25_batch_strang_step)
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
  hipLaunchKernelGGL(k_batch_fold, dim3(1), dim3(64), 0, c->stream, c->d_flag, c->d_counts, fail, acc);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// one Strang step of one run, no host synchronisation (graph-capturable)
static int strang_deferred(mhd25_ctx* c, double* U, double* Bx, double* By, double* Bz, double dt, int* fail,
                           long long* acc, double* eta_out) {
  hipLaunchKernelGGL(k_batch_zero, dim3(1), dim3(64), 0, c->stream, fail, acc, eta_out);
  // entry snapshot with the admissibility test: an inadmissible input makes every attempt of the
  // run fail, so the run is redone individually, which returns status 2
  const double* Bin[3] = {Bx, By, Bz};
  BTRY(entry_snapshot(c, U, c->snapU, Bin, c->saveB));
  BTRY(attempt_deferred(c, U, 0.5 * dt, fail, acc));
  BTRY(mag_to_primitive(c, U, c->rho, c->e, c->u));
  BTRY(step_magnetic_impl(c, c->rho, c->e, c->u, Bx, By, Bz, dt, nullptr));
  if (c->opt.ar && c->opt.C_eta > 0.0) BTRY(extra_max_dev(c, c->eta, c->mp.K, eta_out));
  BTRY(mag_to_conservative(c, c->rho, c->e, c->u, U));
  BTRY(attempt_deferred(c, U, 0.5 * dt, fail, acc));
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
  if (S != b->nbranch) release_graph(b);
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

static int capture(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By, double* const* Bz,
                   const double* dt) {
  release_graph(b);
  std::vector<int> br = assign(b);
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed) != hipSuccess) { b->err = "begin capture"; return -2; }
  hipEventRecord(b->ev_fork, b->cap);
  for (int s = 0; s < b->nbranch; ++s) hipStreamWaitEvent(b->br[s], b->ev_fork, 0);
  int rc = 0;
  for (int r = 0; r < b->nruns && !rc; ++r) {
    mhd25_ctx* c = b->ctx[r];
    c->stream = b->br[br[r]];
    rc = strang_deferred(c, U[r], Bx[r], By[r], Bz[r], dt[r], b->d_fail + r, b->d_acc + 3 * r, b->d_eta + r);
  }
  for (int s = 0; s < b->nbranch; ++s) {
    hipEventRecord(b->ev_join[s], b->br[s]);
    hipStreamWaitEvent(b->cap, b->ev_join[s], 0);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  for (int r = 0; r < b->nruns; ++r) b->ctx[r]->stream = b->main;
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    b->err = "graph capture failed";
    return rc ? rc : -2;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->err = "graph instantiate failed";
    return -2;
  }
  b->captured = true;
  b->cap_dt.assign(dt, dt + b->nruns);
  b->cap_ptr.clear();
  for (int r = 0; r < b->nruns; ++r) {
    b->cap_ptr.push_back(U[r]); b->cap_ptr.push_back(Bx[r]); b->cap_ptr.push_back(By[r]); b->cap_ptr.push_back(Bz[r]);
  }
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

static bool same_capture(const mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                         double* const* Bz, const double* dt) {
  if (!b->captured) return false;
  for (int r = 0; r < b->nruns; ++r) {
    if (b->cap_dt[r] != dt[r]) return false;
    if (b->cap_ptr[4 * r] != U[r] || b->cap_ptr[4 * r + 1] != Bx[r] || b->cap_ptr[4 * r + 2] != By[r] ||
        b->cap_ptr[4 * r + 3] != Bz[r])
      return false;
  }
  return true;
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
  b->allow_capture = false;
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
      hipEventCreateWithFlags(&b->ev_cap, hipEventDisableTiming) != hipSuccess ||
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
  if (b->ev_cap) (void)hipEventDestroy(b->ev_cap);
  if (b->cap) (void)hipStreamDestroy(b->cap);
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
      one.substeps_attempted = 2; one.substeps_accepted = 2;
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
  if (!b->allow_capture) {
    b->err = "the captured multi-branch batch step is disabled: its first GPU run ended in a host segmentation "
             "fault whose cause has not been shown; use mhd25_batch_strang_step_streams";
    return -2;
  }
  if (!same_capture(b, U, Bx, By, Bz, dt)) {
    if (hipStreamSynchronize(b->main) != hipSuccess) { b->err = "sync"; return -2; }
    BTRY(capture(b, U, Bx, By, Bz, dt));
  }
  if (hipGraphLaunch(b->exec, b->main) != hipSuccess) { b->err = "graph launch"; return -2; }
  return finish_step(b, U, Bx, By, Bz, dt, rep);
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
  }
  return 0;
}

// Autotuner.  Per degree p present in the batch, the hydro-stage tile (128 or 256 threads per
// block) is timed with plain launches and HIP events on a scratch copy of the largest run of that
// degree (median of 5 launches after 2 warm-ups); the branch count is min(8, number of runs with at
// least a quarter of the largest run's work, at least 2).  No graph is captured while tuning.
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
    int rbig = -1;
    for (int r = 0; r < b->nruns; ++r)
      if (b->ctx[r]->p == p && (rbig < 0 || b->ctx[r]->mp.K > b->ctx[rbig]->mp.K)) rbig = r;
    if (rbig < 0) continue;
    mhd25_ctx* c = b->ctx[rbig];
    c->stream = b->main;
    const long n5 = 5 * c->mp.K * c->nn;
    // scratch: the run's own stage buffers (idle between steps) hold the copy
    BTRY(dcopy(c, U[rbig], c->S1, n5));
    double best = 1e30;
    const int saved = c->hydro_bs;
    for (int bs : {256, 128}) {
      c->hydro_bs = bs;
      std::vector<float> ms;
      for (int k = 0; k < 7; ++k) {
        BTRY(reset_attempt(c));
        hipEventRecord(e0, b->main);
        BTRY(hydro_stage_a(c, c->S1, c->S1, c->Ust, 0.0, 1.0, 0.25 * dt[rbig]));
        hipEventRecord(e1, b->main);
        if (hipEventSynchronize(e1) != hipSuccess) return -2;
        float t = 0.f;
        hipEventElapsedTime(&t, e0, e1);
        if (k >= 2) ms.push_back(t);
      }
      std::sort(ms.begin(), ms.end());
      const double med = ms[ms.size() / 2];
      if (med < best) { best = med; best_bs[p] = bs; }
    }
    c->hydro_bs = saved;
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
