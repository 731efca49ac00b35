/* mhd25.h -- C ABI of the MI355X (gfx950) library for the Strang-split 2.5D ideal-MHD
 * scheme of Fan & Fu, "Structure-preserving operator splitting for 2.5D ideal MHD with an
 * entropy-stable DGSEM and exactly divergence-free compatible finite elements".
 *
 * Conventions
 *  - Every array argument is a caller-owned, contiguous FP64 (or integer, where stated)
 *    DEVICE pointer, e.g. a torch tensor's data_ptr(); the library never frees it.
 *    Host pointers are used only for the small report / diagnostics structs, as stated.
 *  - Mesh: nx x ny periodic Cartesian elements on [x0,x1]x[y0,y1], element
 *    e = ey*nx + ex.  K = nx*ny.  p = DGSEM degree (1..6), m = compatible magnetic degree
 *    with m in {p-1, p} (section "Magnetic--velocity subflow: compatible finite elements").
 *  - Euler layout U[5][K][p+1][p+1]: (rho, m_x, m_y, m_z, E_mech) at the GLL_p nodes, x index
 *    fastest (section "Hydrodynamic subflow").  rho, e: [K][p+1][p+1]; u: [3][K][p+1][p+1].
 *  - Magnetic layout: every field of the compatible complex is a periodic grid
 *    [ny*(m+1)][nx*(m+1)] of PHYSICAL component values at nodes (eq. hcurl-basis,
 *    eq. hdiv-basis; Piola maps are diagonal on rectangles).  Element (ex,ey) owns grid
 *    columns ex*(m+1)..ex*(m+1)+m and rows ey*(m+1)..ey*(m+1)+m:
 *       B_x, E_y, J_y : GLL_{m+1} in x (last node = neighbour's first) x Gauss_m in y
 *       B_y, E_x, J_x : Gauss_m in x x GLL_{m+1} in y
 *       B_z           : GLL_m x GLL_m (element-local, discontinuous)
 *       E_z, J_z      : GLL_{m+1} x GLL_{m+1} (continuous)
 *  - Calls are stream-ordered on the context's stream.  Calls that return a report or a
 *    decision synchronise that stream.  One context belongs to one stream; concurrent
 *    calls on one context are not allowed.
 *  - Return codes: 0 ok; negative = caller or system error (-1 invalid argument, -2 HIP
 *    error, -3 out of device memory, -4 unsupported degree (p outside 1..6 or m not in
 *    {p-1, p})); positive = numerical outcome with the state left at its value on entry
 *    (1: a hydro substep was not accepted within max_halvings; 2: the input is outside the
 *    admissible set of section "Conservative ideal MHD": a non-finite value, or a non-positive
 *    nodal density or pressure).  The library never aborts; mhd25_last_error() describes
 *    the failure.
 */
#ifndef MHD25_H
#define MHD25_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd25_ctx mhd25_ctx; /* opaque: owns tables, workspace and counters */

typedef struct {
  int32_t nx, ny;           /* elements per direction (>= 1), periodic              */
  double x0, x1, y0, y1;    /* rectangle Omega                                      */
  int32_t p;                /* DGSEM degree, 1..6                                    */
  int32_t m;                /* magnetic degree, p-1 or p                             */
  double gamma;             /* ratio of specific heats (> 1)                         */
  int32_t walls;            /* 0 (default): periodic Omega.  Bit 0 (bit 1): mirror walls normal to x
                             * (to y), section "MHD rotor": Omega is the mirror-doubled image of the
                             * box [x0, (x0+x1)/2] (resp. [y0, (y0+y1)/2]) in that direction, nx (ny)
                             * even, and the caller supplies states with the mirror parities across
                             * the box's walls (rho, p, tangential u even, normal u odd; B_x even and
                             * B_y odd across both kinds of wall; B_z odd across x-normal and even
                             * across y-normal walls).  Every operator is periodic on Omega, which
                             * keeps those parities; the amplitudes of the stabilisers (OE, velocity
                             * OE, A.R.) are taken over the box: the first nx/2 (ny/2) elements of
                             * each row (column) and the box's DOFs, its wall nodes included.    */
} mhd25_mesh_desc;

typedef struct {
  int32_t oe_hydro;         /* hydro oscillation elimination on/off                 */
  int32_t oe_mag;           /* velocity OE on/off                                    */
  int32_t pp;               /* positivity-preserving scaling on/off                  */
  int32_t ar;               /* artificial resistivity on/off                         */
  double s_H, s_M;          /* OE scale factors (paper: 0.02)                        */
  double C_s, C_eta;        /* A.R. sensor response and maximum (paper: 5, 0.2)      */
  int32_t iface_flux;       /* 0: local Lax-Friedrichs (the scheme), 1: the EC flux  */
  int32_t max_halvings;     /* reject-and-halve depth budget (default 10)            */
  int32_t reduced_2d2v;     /* 2D2V reduced system (section "Numerical experiments"): the
                             * caller guarantees u_z = 0 and B_z = 0; the magnetic substep then
                             * neither reads nor writes u_z and B_z and skips the identically
                             * zero in-plane E and J (results equal the general path's). Default 0 */
  int32_t strang_order;     /* 0 (default): H(dt/2) M(dt) H(dt/2), the composition the paper states
                             * (eq. strang-composition, Algorithm "Strang split MHD step");
                             * 1: M(dt/2) H(dt) M(dt/2), the magnetic-outer composition, whose
                             * results reproduce the magnitudes of the paper's temporal table */
} mhd25_options;

typedef struct {
  int32_t substeps_attempted; /* hydro substep attempts (including rejected ones)   */
  int32_t substeps_accepted;
  int32_t max_depth;          /* deepest halving level reached                      */
  int32_t status;             /* return code of the call                            */
  int64_t n_rho_limited;      /* elements with density scaling, summed over stages  */
  int64_t n_p_limited;        /* elements with pressure scaling                     */
  int64_t n_collapsed;        /* elements collapsed to their average                */
  double eta_max;             /* max artificial-resistivity coefficient (last M stage) */
  double dt;                  /* step size of the call                              */
} mhd25_report;

/* Defaults: all stabilisation off, paper constants, LLF interfaces, 10 halvings. */
void mhd25_default_options(mhd25_options* opt);

/* Create a context for one mesh.  `hip_stream` is a hipStream_t (NULL = default stream).
 * Allocates all device workspace (about 12 state-sized arrays).  Returns 0, or -1 for a null
 * pointer, nx or ny < 1, an empty domain, gamma <= 1, nx * ny * (m + 1) above 2^31 - 2^16 or
 * nx * ny * (p + 1)^2 nodes at or above 2^29 (both far beyond device memory) or invalid options; -4 for p outside 1..6 or m not in {p - 1, p}; -3 when host or device memory runs out. */
int mhd25_init(const mhd25_mesh_desc* mesh, const mhd25_options* opt, void* hip_stream, mhd25_ctx** out);
void mhd25_destroy(mhd25_ctx* ctx);
/* Replace the options of an existing context (host-side only). */
int mhd25_set_options(mhd25_ctx* ctx, const mhd25_options* opt);
const char* mhd25_last_error(const mhd25_ctx* ctx);

/* L_E: mass-inverted DGSEM operator (eq. euler-nodal-index / eq. euler-semidiscrete):
 * entropy-conservative flux differencing (eq. euler-chandrashekar-flux,
 * eq. euler-volume-residual) with LLF interfaces (eq. euler-lf-flux).
 * U, dUdt: [5][K][p+1][p+1]; dUdt is overwritten. */
int mhd25_rhs_hydro(mhd25_ctx* ctx, const double* U, double* dUdt);

/* Stage map P = P_PP o P_OE (eq. euler-stage-map) applied in place to a raw stage candidate
 * U with stage step tau.  `flags` (device, [K] uint8, may be NULL) receives bit0 density
 * limited, bit1 pressure limited, bit2 collapsed.  Returns 0; does not check admissibility. */
int mhd25_hydro_stage_map(mhd25_ctx* ctx, double* U, double tau, uint8_t* flags);

/* Algorithm "Hydrodynamic Euler substep": SSP-RK(3,3) (eq. euler-ssprk33) with P after every
 * raw stage; a raw stage whose element average is inadmissible rejects the attempt, which
 * is replaced by two attempts of tau/2 (recursively, depth <= max_halvings).  U in place.
 * `rep` (host, may be NULL) is filled.  Returns 0, 1 (not accepted; U unchanged), 2 (U has a
 * non-finite value or a non-positive nodal rho or p; U unchanged, nothing attempted) or <0. */
int mhd25_hydro_substep(mhd25_ctx* ctx, double* U, double tau, mhd25_report* rep);

/* L_M: mass-inverted magnetic-velocity operator with J and E eliminated (eq. magnetic-dae):
 * weak-curl current (eq. mag-current-proj), Ohm-law electric field (eq. mag-electric-proj),
 * strong curl update, Lorentz load as the transpose of the coupling form, Ohmic heating.
 * rho frozen, eta ([K], may be NULL = ideal) frozen.  Outputs overwritten:
 * de [K][p+1]^2, du [3][K][p+1]^2, dBx/dBy/dBz magnetic grids. */
int mhd25_rhs_magnetic(mhd25_ctx* ctx, const double* rho, const double* u, const double* Bx,
                       const double* By, const double* Bz, const double* eta, double* de, double* du,
                       double* dBx, double* dBy, double* dBz);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mhd25_rhs_magnetic with the same arguments, kernels
 * and results, whose workspace (the six reconstructed J, E grids and the per-element loads) is a
 * fixed file-scope device array of 32 MiB per device instead of the context's workspace.  The
 * call allocates nothing (its address is resolved once per device by mhd25_init).  The mesh must
 * need at most 32 MiB: 8 (6 G + K (2 (m+2)(m+1) + (m+2)^2)) bytes with G = K (m+1)^2 (up to
 * 211 x 211 elements at m = 2, 161 x 161 at m = 3); larger meshes return -1 before any device
 * work.  Every call on a device shares that device's array: calls that overlap on one device
 * (different streams, threads or contexts) race and must be serialised by the caller.  No
 * entry of the array needs to start at zero (each is written before it is read).  Returns 0,
 * -1 (null pointer or mesh above the limit) or -2 (no context was created on the current device,
 * or a launch failed). */
int mhd25_rhs_magnetic_noalloc(mhd25_ctx* ctx, const double* rho, const double* u, const double* Bx,
                               const double* By, const double* Bz, const double* eta, double* de,
                               double* du, double* dBx, double* dBy, double* dBz);

/* Reconstructed current and electric field (eq. mag-current-proj, eq. mag-electric-proj):
 * J6 = six magnetic grids (J_x, J_y, J_z, E_x, E_y, E_z) in that order, overwritten. */
int mhd25_reconstruct_JE(mhd25_ctx* ctx, const double* u, const double* Bx, const double* By,
                         const double* Bz, const double* eta, double* JE6);

/* Artificial-resistivity coefficient eta_K (eq. magnetic-ar-sensor, eq. magnetic-ar-coefficient)
 * of the state (rho, u, B).  eta: [K], overwritten. */
int mhd25_ar_eta(mhd25_ctx* ctx, const double* rho, const double* u, const double* Bx, const double* By,
                 const double* Bz, double* eta);

/* Velocity OE map (eq. magnetic-oe-sensor .. eq. magnetic-oe-map) applied in place to (u, e)
 * of a raw magnetic stage with step tau; B is read for the rate. */
int mhd25_velocity_oe(mhd25_ctx* ctx, double tau, const double* rho, double* u, double* e,
                      const double* Bx, const double* By, const double* Bz);

/* Algorithm "Magnetic-velocity substep": eta frozen at entry (when ar is on), SSP-RK(3,3)
 * (eq. magnetic-ssprk33) with the velocity OE after every raw stage.  e, u, B in place.
 * Returns 0, 2 (a non-finite value, or a non-positive nodal rho or e, in the input; nothing is
 * modified) or <0.  The entry test synchronises the stream once. */
int mhd25_step_magnetic(mhd25_ctx* ctx, const double* rho, double* e, double* u, double* Bx,
                        double* By, double* Bz, double tau, mhd25_report* rep);

/* Nodal variable exchange (section "Local variable exchange"). */
int mhd25_to_primitive(mhd25_ctx* ctx, const double* U, double* rho, double* e, double* u);
int mhd25_to_conservative(mhd25_ctx* ctx, const double* rho, const double* e, const double* u, double* U);

/* Algorithm "Strang split MHD step": H(dt/2) -> exchange -> M(dt) -> exchange -> H(dt/2), or with
 * strang_order = 1 exchange -> M(dt/2) -> exchange -> H(dt) -> exchange -> M(dt/2) -> exchange.
 * U and B in place.  Returns 0, 1 (a hydro substep not accepted within max_halvings), 2 (U or B
 * has a non-finite value, or U a non-positive nodal rho or p) or <0; on a positive return U and
 * B are restored to their entry values.  The entry test is folded into the entry snapshot. */
int mhd25_strang_step(mhd25_ctx* ctx, double* U, double* Bx, double* By, double* Bz, double dt,
                      mhd25_report* rep);

/* Time step from the positivity CFL: dt = cfl / max_{K,q} (2p+1)[(|u_x|+c_f)/hx + (|u_y|+c_f)/hy],
 * c_f = sqrt((gamma p + |B|^2)/rho) with B at the GLL_p nodes.  dt written to *dt (host).
 * Returns 2 when the maximum is not a positive finite number (an inadmissible state). */
int mhd25_cfl_dt(mhd25_ctx* ctx, const double* U, const double* Bx, const double* By, const double* Bz,
                 double cfl, double* dt);

/* In-plane field (-d_y A_h, d_x A_h) of a potential A_h on the E_z/J_z grid (initial data,
 * section "Advected MHD vortex"). */
int mhd25_B_from_potential(mhd25_ctx* ctx, const double* A, double* Bx, double* By);

/* Diagnostics (host out[6]): mass = sum M rho, mechanical energy sum M E_mech,
 * magnetic energy (B,B)_B / 2, ||div B||_{L2}, min nodal rho, min nodal p.  Over the whole mesh:
 * on a mirror-walled mesh the sums are those of the box times the number of images (2 or 4), the
 * L2 norm the box's times the square root of that number. */
int mhd25_diagnostics(mhd25_ctx* ctx, const double* U, const double* Bx, const double* By,
                      const double* Bz, double* out6);

/* Physical coordinates (x, y) of the nodes of one node set (section "Spatial preparation";
 * element map x = x_K + (xi + 1) h / 2 per direction).  space 0: the GLL_p element nodes,
 * x and y [K][p+1][p+1]; 1: B_x grid (GLL_{m+1} x Gauss_m); 2: B_y grid (Gauss_m x GLL_{m+1});
 * 3: B_z grid (GLL_m x GLL_m); 4: W grid of E_z, J_z (GLL_{m+1}^2); 5: N_x grid of E_x, J_x
 * (Gauss_m x GLL_{m+1}); 6: N_y grid of E_y, J_y (GLL_{m+1} x Gauss_m); grids [ny(m+1)][nx(m+1)].
 * Grid node (gy, gx) is local node (gx mod (m+1), gy mod (m+1)) of element (gx/(m+1), gy/(m+1));
 * a node shared by two elements is the first local node of the right / upper one.  x, y: device
 * FP64 arrays, overwritten.  Returns 0 or -1 (null pointer, space outside 0..6). */
int mhd25_node_coords(mhd25_ctx* ctx, int32_t space, double* x, double* y);

/* Connectivity of the conforming periodic mesh (section "Spatial preparation") as used by the
 * kernels.  elem_nbr: device int32 [K][4], the neighbour across the left, right, bottom and top
 * face.  dof_maps (device int32, may be NULL), concatenated:
 *   face map [K][4][p+1]: for face f (left, right, bottom, top) and face node k (k indexes y on
 *     the left / right faces, x on the bottom / top faces) the index e' (p+1)^2 + q' (q' = j (p+1) + i)
 *     of the neighbour's node at the same point;
 *   then [K][n_s] local-to-global grid indices of the six magnetic node sets B_x ((m+2)(m+1)),
 *     B_y ((m+1)(m+2)), B_z ((m+1)^2), W ((m+2)^2), N_x ((m+1)(m+2)), N_y ((m+2)(m+1)), each in
 *     local order [j][i], i fastest, i in x.
 * Total length K (4(p+1) + 4(m+1)(m+2) + (m+1)^2 + (m+2)^2).  Returns 0, -1 (null pointer, or an
 * index beyond the int32 range). */
int mhd25_get_maps(mhd25_ctx* ctx, int32_t* elem_nbr, int32_t* dof_maps);

/* Per-element decision flags of the last stage map applied (device [K] uint8 copied to the
 * host buffer `host_flags` of length n >= K).  Bit-exact comparisons use these. */
int mhd25_decisions(const mhd25_ctx* ctx, uint8_t* host_flags, int64_t n);

/* Vector-Jacobian products (stage recomputation, no stored Jacobians).
 * Hydro: Ubar = (dL_E/dU)^T cot with the LLF max/abs branches taken at U.  Ubar overwritten.
 * Magnetic: VJP of L_M with rho and eta frozen; e does not enter L_M (ebar = 0). */
int mhd25_rhs_hydro_vjp(mhd25_ctx* ctx, const double* U, const double* cot, double* Ubar);
int mhd25_rhs_magnetic_vjp(mhd25_ctx* ctx, const double* rho, const double* u, const double* Bx,
                           const double* By, const double* Bz, const double* eta, const double* de_cot,
                           const double* du_cot, const double* dBx_cot, const double* dBy_cot,
                           const double* dBz_cot, double* u_bar, double* Bx_bar, double* By_bar,
                           double* Bz_bar);

/* Kernel timing on the context stream with HIP events (off by default).  Kernel ids: 0 the hydro
 * stage kernel (L_E + SSP combine + statistics), 1 the hydro stage map (OE + PP), 2 the magnetic
 * update, 3 the velocity-OE projection, 4 the velocity-OE preparation, 5 the E loads, 6 the
 * velocity-OE sensor, 7 the J loads, 8 the gathers, 9 the A.R. traces.  mhd25_timing_read returns
 * the launches and summed ms of one kernel since its last read and resets them; another id or a
 * NULL pointer returns -1. */
int mhd25_timing_enable(mhd25_ctx* ctx, int32_t on);
int mhd25_timing_read(mhd25_ctx* ctx, int32_t kernel_id, int64_t* launches, double* total_ms);

/* ---- Batched ensemble of independent runs (uneven meshes and degrees) ---- */
typedef struct mhd25_batch mhd25_batch;
/* Create a batch of nruns runs, each with its own mesh; options shared. */
int mhd25_batch_create(const mhd25_mesh_desc* runs, int32_t nruns, const mhd25_options* opt,
                       void* hip_stream, mhd25_batch** out);
void mhd25_batch_destroy(mhd25_batch* b);
const char* mhd25_batch_last_error(const mhd25_batch* b);
/* One Strang step of every run (extension: batched ensembles) by run-table launches: every launch
 * of the step covers all runs of one degree group, its blocks split into consecutive per-run
 * ranges, so one step issues about 150 launches for 64 runs; each degree group's launches go to a
 * branch stream of its own (between fork and join events on hip_stream), so the groups overlap.
 * The per-run arguments are uploaded once per set of pointers and steps (a change of either
 * rebuilds the plan: one host-to-device copy).  With mhd25_batch_graph(b, 1) the step instead
 * replays a HIP graph of those launches, captured in order on one stream of the batch.  U, Bx, By, Bz: host arrays of nruns device pointers; dt: host [nruns]; rep:
 * host [nruns] (may be NULL).  Runs whose hydro substep needs a halving, or whose input is
 * inadmissible, are restored and re-done individually with mhd25_strang_step.  Results equal
 * mhd25_strang_step of each run bit for bit.  Returns 0, or the first nonzero run status (1, 2, <0). */
int mhd25_batch_strang_step(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                            double* const* Bz, const double* dt, mhd25_report* rep);
/* One Strang step of every run without a graph: each run's deferred step (no host read inside)
 * is launched directly on its branch stream, between a fork event on the context stream and join
 * events that the context stream waits on.  U, Bx, By, Bz: host arrays of nruns device pointers;
 * dt: host [nruns]; rep: host [nruns] (may be NULL).  Runs whose hydro substep needs a halving, or
 * whose input is inadmissible, are re-done individually with mhd25_strang_step.  Returns 0, or
 * the first nonzero run status (1, 2 or <0). */
int mhd25_batch_strang_step_streams(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                                    double* const* Bz, const double* dt, mhd25_report* rep);
/* Graph mode of mhd25_batch_strang_step: 1 = capture the run-table step into a HIP graph on the
 * batch's stream (once per plan) and replay it; 0 = plain launches; -1 = release the graph and use
 * plain launches.  Returns 0 or -1. */
int mhd25_batch_graph(mhd25_batch* b, int32_t capture_or_replay);
/* Sequential reference: the same step run by run with the plain per-run kernels. */
int mhd25_batch_strang_step_sequential(mhd25_batch* b, double* const* U, double* const* Bx,
                                       double* const* By, double* const* Bz, const double* dt,
                                       mhd25_report* rep);

/* Tuning knobs of the batch: number of concurrent branch streams of the streams step (1..8; <= 0
 * leaves it) and the hydro-stage tile (128 or 256 threads per block) for runs of degree p (p <= 0:
 * all runs).  Invalidates the run-table plan and its graph. */
int mhd25_batch_set_tuning(mhd25_batch* b, int32_t branches, int32_t p, int32_t hydro_bs);
/* Autotuner: per degree present, times the hydro-stage tiles (128 / 256 threads per block) with
 * plain launches on a scratch copy of the largest run of that degree (the given states are not
 * modified), sets the branch count to min(8, max(2, number of runs with >= 1/4 of the largest
 * run's work)), and appends the choice to the JSON-lines file `cache_path` (may be NULL); a line
 * for the same run set is reused without timing.  *best_branches (host, may be NULL) receives
 * the branch count. */
int mhd25_batch_autotune(mhd25_batch* b, double* const* U, double* const* Bx, double* const* By,
                         double* const* Bz, const double* dt, const char* cache_path, int32_t* best_branches);

#ifdef __cplusplus
}
#endif
#endif /* MHD25_H */
