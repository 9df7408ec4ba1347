/*
 * hrlb.h -- C ABI of libhrlb, the MI355X (gfx950) time step of the mixed-quadrature
 * lattice Boltzmann solver for 3D Couette flow of Ambrus & Sofonea, "Half-range lattice
 * Boltzmann models for the simulation of Couette flow using the Shakhov collision term"
 * (arXiv:1702.01335).
 *
 * Problem (Sec. III): plates at x = -L/2 and x = +L/2 (L = 1) move with -u_w and +u_w
 * along y and are kept at T_w; by the centre-line symmetry the solver holds the half
 * channel 0 <= x <= L/2 in S nodes (App. A.4), with bounce-back at x = 0 and diffuse
 * reflection at x = L/2.  The velocity set is the product of a half-range Gauss-Hermite
 * rule on x (2 Qx nodes) and full-range rules on y (Qy) and z (Qz): V = 2 Qx Qy Qz
 * discrete velocities, flat index v = (i Qy + j) Qz + k, nodes ascending on each axis.
 * Collision: Shakhov (BGK when Pr = 1), Eq. boltz, with the Hermite-projected
 * equilibrium of Sec. III and tau from a power-law or Sutherland viscosity.  Space: WENO-5
 * (App. A.3) or second-order upwind on the tanh-stretched grid (App. A.2).  Time: TVD RK3
 * (App. A.1).
 *
 * Conventions
 *  - Every function returns HRLB_OK (0) or a negative status; nothing throws or aborts.
 *    hrlb_last_error() gives a message for the calling thread's last failure.
 *  - Device memory is owned by the caller.  The library keeps raw pointers into the
 *    caller's state and work buffers for the lifetime of an hrlb_sim and never frees them.
 *    Host handles (hrlb_quad, hrlb_sim) are owned by the library and released by the
 *    matching *_free call.
 *  - All device work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *    NULL = the null stream).  Only hrlb_residual synchronises that stream.
 *  - Population arrays are FP64, layout [B][S][V] (instance, node, velocity), v fastest.
 */
#ifndef HRLB_H
#define HRLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HRLB_OK 0
#define HRLB_EINVAL (-1)   /* invalid argument (sizes, parameters, null pointers)        */
#define HRLB_ENOMEM (-2)   /* caller buffer smaller than hrlb_state_bytes requires        */
#define HRLB_EHIP (-3)     /* a HIP runtime call failed; message holds hipGetErrorString  */
#define HRLB_ENUMERIC (-4) /* n <= 0, T <= 0 or a non-finite moment met during a step, or a
                              time step beyond the RK3 stability limit (hrlb_init_state)   */

#define HRLB_LAW_POWER 0      /* mu = kn T^omega  -> tau = kn T^(omega-1) / n  (Eq. mw_tau for omega = 1) */
#define HRLB_LAW_SUTHERLAND 1 /* mu = kn sqrt(T)(1+S)/(1+S/T) -> Eq. sutherland_tau with kn = 1/(delta sqrt 2) */
#define HRLB_LAW_LOWMACH 2    /* constant tau = kn / sqrt(2), kn = k: the linearised regime of Sec. IV, Eq. knLuo */

#define HRLB_SCHEME_UPWIND2 0 /* second-order upwind fluxes                                  */
#define HRLB_SCHEME_WENO5 1   /* epsilon-free WENO-5, Eqs. weno5_flux..weno_sigma, Table II  */
#define HRLB_SCHEME_LINEAR5 2 /* the WENO-5 candidate fluxes with the ideal weights (linear fifth order) */

/* Physical and numerical parameters of one Couette instance (non-dimensional, Sec. II.B). */
typedef struct hrlb_params {
  double kn;       /* rarefaction: mu(T = 1) = kn, i.e. Kn of Sec. V, 1/(delta sqrt 2) of Sec. VI; > 0 */
  double u_w;      /* wall speed; the wall at x = +L/2 moves with +u_w along y                       */
  double T_w;      /* wall temperature (> 0)                                                          */
  double n0;       /* initial density of the equilibrium start (> 0)                                 */
  double pr;       /* Prandtl number of the Shakhov model (> 0); 1 = BGK                              */
  double omega;    /* viscosity index of HRLB_LAW_POWER                                               */
  double suth_S;   /* Sutherland constant S / T_ref of HRLB_LAW_SUTHERLAND (>= 0)                      */
  double A;        /* tanh stretching of Eq. stretch, 0 <= A < 1; 0 = equidistant nodes               */
  double dt;       /* time step (> 0)                                                                 */
  int law;         /* HRLB_LAW_*                                                                      */
  int collisionless; /* nonzero: drop the collision term (1/tau = 0)                                 */
} hrlb_params;

typedef struct hrlb_quad hrlb_quad;
typedef struct hrlb_sim hrlb_sim;
typedef struct hrlb_batch hrlb_batch;

/* Message for the calling thread's last failed call ("" if none). Owned by the library. */
const char* hrlb_last_error(void);

/*
 * trace_status -- whether the library emits roctx ranges.  With HRLB_TRACE set to anything
 * but "" or "0" when the library is first used, and the roctx library
 * (librocprofiler-sdk-roctx) loadable, every call below that enqueues work pushes a range
 * named after itself ("hrlb_step", "hrlb_moments", ...), each graph launch one more ("RK3
 * steps (graph launch)" for eight steps, "RK3 step (graph launch)" for one), and an eager
 * step one per launch ("closure",
 * "RK3 stage 1".."3"); a rocprofv3 --marker-trace run shows them beside the kernels.  The
 * ranges cover the host-side enqueue, not the kernels' execution.  *enabled = 1 when ranges
 * are emitted, else 0.  Errors: HRLB_EINVAL for a NULL pointer.
 */
int hrlb_trace_status(int* enabled);

/*
 * init_quadrature -- host-side velocity set and Hermite projection tables (Sec. III:
 * HHLB(Nx;Qx) x HLB(Ny;Qy), here with a third full-range factor HLB(Nz;Qz) on z).
 *   Qx: nodes per x semi-axis, 1..128; Nx: half-range expansion order, 0..min(Qx-1, 8)
 *   (the paper uses Nx = min(6, Qx-1)).  Qy, Qz: full-range nodes, 1..16; Ny <= Qy-1,
 *   Nz <= Qz-1 (the paper uses N = Q-1).  No device work.
 *   Errors: HRLB_EINVAL on out-of-range orders or out == NULL.
 */
int hrlb_init_quadrature(int Qx, int Nx, int Qy, int Ny, int Qz, int Nz, hrlb_quad** out);
/*
 * init_quadrature_reduced -- the paper's own velocity set HHLB(Nx;Qx) x HLB(Ny;Qy) with p_z
 * integrated out (Sec. III: the reduced distributions phi = int f dp_z and chi = int f p_z^2
 * dp_z of Eq. reduced_def, evolved by Eq. boltz_red with phi^eq of Eq. phieq, chi^eq =
 * T phi^eq and the reduced Shakhov factors of Eq. sred_def; at the wall chi_w = T_w phi_w,
 * App. A.4).  A sim built on it carries V = 4 Qx Qy populations per node, flat index
 * v = (i Qy + j) 2 + c with c = 0 for phi and c = 1 for chi; everything else (step,
 * moments with u_z = q_z = P_xz = P_yz = 0 and P_zz = sum chi, residual, batches, launch
 * shapes) is as for the explicit set.  hrlb_quad_nodes has no axis 2 for it, and
 * hrlb_seed_state rejects its sims.  Orders as for hrlb_init_quadrature; HRLB_EINVAL
 * otherwise.
 */
int hrlb_init_quadrature_reduced(int Qx, int Nx, int Qy, int Ny, hrlb_quad** out);
void hrlb_quad_free(hrlb_quad* q);

/* Number of populations per node: V = 2 Qx Qy Qz (4 Qx Qy for the reduced model). */
int hrlb_quad_size(const hrlb_quad* q, int* V);

/*
 * Nodes and weights of one axis (0 = x: 2 Qx values, ascending, weights summing to 1;
 * 1 = y: Qy values; 2 = z: Qz values).  Host buffers of the axis' length.
 */
int hrlb_quad_nodes(const hrlb_quad* q, int axis, double* nodes, double* weights);

/*
 * state_bytes -- device bytes the caller allocates for `batch` instances of S nodes:
 *   *state_bytes: three population arrays [batch][S][V] (the step's F_l and two RK
 *                 stage buffers); *work_bytes: tables, moment partials, per-node closure,
 *                 wall densities, residual partials and fault flags.
 * Both buffers must be 256-byte aligned (torch allocations are).  One instance's
 * populations, S * V * 8 bytes, must stay below 4 GiB (HRLB_EINVAL otherwise); the
 * batch as a whole has no such limit.
 */
int hrlb_state_bytes(const hrlb_quad* q, int S, int batch, size_t* state_bytes, size_t* work_bytes);

/*
 * init_state -- bind buffers and write the initial state of `batch` instances that
 * share the velocity set `q`, the node count S (>= 3) and the flux scheme.
 *   params[b]: per-instance parameters (host array of `batch` entries).
 *   d_state, d_work: caller device buffers of at least the hrlb_state_bytes sizes.
 *   stream: hipStream_t all work of this sim is enqueued on.
 *   d_perturb: NULL, or a device array r[batch][S][V]; the initial state is
 *     F = n0 F^eq(u = 0, T = T_w) (1 + eps r) with F^eq the discrete equilibrium at rest.
 *     (The paper does not state its initial condition; equilibrium at rest is the
 *     library's reading.)
 * The quadrature handle must outlive the sim.
 * Errors: HRLB_EINVAL (S < 3, batch < 1, dt <= 0, kn <= 0, T_w <= 0, n0 <= 0, pr <= 0,
 *   A outside [0, 1), unknown law or scheme, one instance's S * V * 8 bytes not below
 *   4 GiB), HRLB_ENUMERIC (a time step beyond the stability limit of the explicit TVD RK3
 *   scheme, Eq. rk3: Courant number max|p_x| dt / min dx above 0.628 for second-order upwind
 *   or 1.434 for the linear fifth-order form, the limits of the amplification factor
 *   1 + z + z^2/2 + z^3/6 over the Fourier symbols of these linear schemes; above 2 for
 *   WENO-5, whose nonlinear weights the paper runs at up to 1.65 (Table III), as a guard;
 *   or dt / tau above 2.512, the limit on the negative real axis, at the initial state
 *   (n0, T_w)), HRLB_ENOMEM (buffers too small), HRLB_EHIP.
 */
int hrlb_init_state(const hrlb_quad* q, int S, int scheme, const hrlb_params* params, int batch,
                    void* d_state, size_t state_bytes, void* d_work, size_t work_bytes, void* stream,
                    const double* d_perturb, double eps, hrlb_sim** out);
void hrlb_sim_free(hrlb_sim* sim);

/*
 * step -- enqueue `nsteps` TVD RK3 steps (Eq. rk3) of every instance.  Each stage
 * rebuilds the ghost nodes and the wall density from its own input (App. A.4), takes the
 * moments of Eq. qdef, the relaxation time and the Shakhov target (Eqs. phieq, sdef) and
 * advances F by L[F] of Eq. L_def.  Asynchronous; a numerical fault surfaces at the next
 * hrlb_residual.  Errors: HRLB_EINVAL (nsteps < 0), HRLB_EHIP.
 */
int hrlb_step(hrlb_sim* sim, int nsteps);

/*
 * moments -- enqueue the per-node moments of the current state (Eq. qdef, m = 1) into
 * the device array d_out[batch][S][14]: n, u_x, u_y, u_z, T, P_xx, P_yy, P_zz, P_xy,
 * P_xz, P_yz, q_x, q_y, q_z (P_ab is the paper's pressure tensor T_ij, T = tr P / 3n).
 */
int hrlb_moments(hrlb_sim* sim, double* d_out);

/*
 * residual -- synchronise the stream and write to the host array h_out[batch] the
 * residual of the last completed step, R = ||F_{l+1} - F_l||_2 / (dt ||F_l||_2) over the
 * fluid nodes (a relative rate per unit time; the paper leaves the stopping rule open).
 * Returns HRLB_ENUMERIC if any instance met n <= 0, T <= 0 or a non-finite moment since
 * init (h_out is still written; the flags stay set).  Before any step h_out is 0.
 */
int hrlb_residual(hrlb_sim* sim, double* h_out);

/* Copy the current state (interior nodes, [batch][S][V]) to / from a caller device array
 * (enqueued on the sim's stream).  set_state also recomputes the moment partials. */
int hrlb_get_state(hrlb_sim* sim, double* d_out);
int hrlb_set_state(hrlb_sim* sim, const double* d_in);

/*
 * seed_state -- warm start: overwrite the state with populations built from a moment
 * table d_table[batch][S][14] (device, caller-owned, the column order of hrlb_moments).
 * Each node gets the projected discrete equilibrium at its n, u, T (Sec. III) times
 * 1 + Pi_ab xi_a xi_b / (2 n T^2) + (xi^2 / (5T) - 1) xi.q / (n T^2), with xi = p - u and
 * Pi = P - n T I: the heat-flux polynomial is that of the Shakhov factor (Eq. sdef) with
 * 1 - Pr replaced by 1, and the stress term carries the pressure deviator.  With
 * equilibrium orders >= 6 on every axis the seed has exactly the table's moments.
 * preserve_mass != 0 scales each instance's seed by one factor so that its mass
 * sum_s n_s dx_s equals that of the equilibrium start, n0 times the half-channel length:
 * the scheme conserves mass (App. A.4), so the steady state reached depends on it.
 * Fallback: an instance whose table has a non-finite entry, n <= 0 or T <= 0 at any node
 * is seeded with the equilibrium at rest (n0, u = 0, T_w) as hrlb_init_state does;
 * h_fallback[batch] (host, may be NULL) receives 1 for those instances.  Recomputes the
 * moment partials, clears the numeric-fault flags and synchronises the stream.
 * Errors: HRLB_EINVAL (NULL sim or table), HRLB_EHIP.
 */
int hrlb_seed_state(hrlb_sim* sim, const double* d_table, int preserve_mass, int* h_fallback);

/*
 * free_molecular_state -- overwrite the state with the free-molecular steady state of the
 * diffuse walls, the collisionless limit of Sec. IV (its shear stress is T_xy^bal of
 * Eq. Txy_bal): at every node, the populations with p_x < 0 are n0 times the discrete wall
 * Maxwellian (u_w, T_w) and those with p_x > 0 are their bounce-back images (Eq. widetildei),
 * i.e. the Maxwellian of the wall at -L/2.  It is a fixed point of the collisionless step, and
 * the start from which runs at large Kn settle fastest.  Recomputes the moment partials and
 * clears the numeric-fault flags and residuals; enqueued on the sim's stream.
 * Errors: HRLB_EINVAL (NULL sim), HRLB_EHIP.
 */
int hrlb_free_molecular_state(hrlb_sim* sim);

/*
 * Launch shape of the stage kernel: `cells` nodes marched per thread (1..4096; 0 = the
 * library's default) and `waves` 64-lane waves per workgroup along v (1..4; 0 = default).
 * Any shape gives the same result up to the summation order of the moment partials.
 */
int hrlb_set_launch(hrlb_sim* sim, int cells, int waves);
int hrlb_get_launch(const hrlb_sim* sim, int* cells, int* waves);

/*
 * autotune -- choose the stage kernel's launch shape for this sim's (velocity set, S,
 * batch, scheme) by timing candidate shapes (cells in 2..128, waves in 1..4) with HIP
 * events over `probe_steps` graph-replayed steps each, and select the fastest.  The probe
 * steps are real steps: they advance the state.  If `cache_path` names a file holding an
 * entry for this shape (JSON lines written by an earlier call), that entry is used and
 * nothing is timed (*best_ms = -1); otherwise the result is appended to the file.
 * Synchronises the stream.  Errors: HRLB_EINVAL, HRLB_EHIP.
 */
int hrlb_autotune(hrlb_sim* sim, int probe_steps, const char* cache_path, int* best_cells, int* best_waves,
                  double* best_ms);

/*
 * Graph mode: when on, hrlb_step replays HIP graphs on the sim's stream instead of
 * launching the kernels one by one: one holding eight RK3 steps (48 launches) for each
 * whole eight of nsteps, one holding a single step (six launches) for the rest, each
 * captured on a private stream when first needed and again after a launch-shape change.
 * Results are identical to the eager path.  Timing mode uses the eager path.
 */
int hrlb_set_graph(hrlb_sim* sim, int on);

/*
 * Optional per-kernel timing: when on, hrlb_step brackets every launch with HIP events on
 * the sim's stream; hrlb_get_timing synchronises and returns the accumulated device time
 * in ms and launch counts of [0] the stage kernel, [1] the closure kernel.  Turning it on
 * resets the accumulators.
 */
int hrlb_set_timing(hrlb_sim* sim, int on);
int hrlb_get_timing(hrlb_sim* sim, double* ms, long long* launches);
/* The same accumulators per RK3 stage (Eq. rk3): ms[4] and launches[4] receive the stage
 * kernel's time and launch count of stages 1, 2 and 3, then the closure kernel's. */
int hrlb_get_stage_timing(hrlb_sim* sim, double* ms, long long* launches);

/*
 * Batches: advance several sims -- each a group of instances sharing one velocity set,
 * node count and scheme, the groups differing in any of them -- together, with one
 * launch per kernel per RK3 stage.  The launches read device-side tables of
 * (group, instance, velocity block, node chunk) tiles and of closure work items (one block
 * each; retired instances drop out of both tables, so blocks past the live counts return
 * at once); one RK3
 * step of the whole batch, and eight steps for runs of eight or more, are captured as HIP
 * graphs on first use and replayed.  Results
 * are those of stepping every sim alone with the same launch shape, bit for bit.
 *
 * batch_bytes: device bytes of the batch's tables (caller-owned, 256-byte aligned).
 * batch_create: `cells` nodes per thread and `waves` waves per workgroup for every group
 *   (each sim's launch shape is set to it); enqueues on `stream` and synchronises it.  The
 *   sims must stay alive and must not be stepped on their own while the batch is in use.
 * batch_step: nsteps RK3 steps of every active instance (asynchronous).
 * batch_residual: synchronise; h_out[i] is the residual of concatenated instance i (the
 *   instances of sims[0], then sims[1], ...); HRLB_ENUMERIC as for hrlb_residual.
 * batch_set_active: active[i] = 0 retires instance i (its state stops advancing; it can be
 *   re-activated); rewrites the tile table; synchronises the stream.
 * Errors: HRLB_EINVAL, HRLB_ENOMEM, HRLB_EHIP, HRLB_ENUMERIC.
 */
int hrlb_batch_bytes(hrlb_sim* const* sims, int nsims, int cells, int waves, size_t* bytes);
int hrlb_batch_create(hrlb_sim* const* sims, int nsims, int cells, int waves, void* d_work, size_t work_bytes,
                      void* stream, hrlb_batch** out);
int hrlb_batch_step(hrlb_batch* batch, int nsteps);
int hrlb_batch_residual(hrlb_batch* batch, double* h_out);
int hrlb_batch_set_active(hrlb_batch* batch, const int* active);
int hrlb_batch_info(const hrlb_batch* batch, int* ntiles, int* nitems, int* grid_stage, int* grid_closure);
void hrlb_batch_free(hrlb_batch* batch);

/*
 * step_noalloc -- for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hrlb_init_state's tables,
 * then `nsteps` RK3 steps as hrlb_step takes them, then optionally hrlb_moments, on the
 * caller's populations, with every table, moment partial, closure record and flag in a fixed
 * device array of HRLB_SCRATCH_BYTES that the library holds on each GPU it runs on until the
 * process ends.  No hipMalloc, hipFree or other allocating device call is made.
 *   q, S, scheme, params, batch: as for hrlb_init_state.
 *   d_state: caller device buffer of hrlb_state_bytes' state size (256-byte aligned); its
 *     first array [batch][S][V] holds F_l on entry and F_{l+nsteps} on return, the other
 *     two are overwritten.
 *   d_moments: NULL, or a device array [batch][S][14] that receives the moments of the
 *     result in hrlb_moments' column order.
 *   stream: hipStream_t everything is enqueued on.
 * The launch shape is the library's default; the results equal those of hrlb_init_state,
 * hrlb_set_state with the same populations, hrlb_step(nsteps) eagerly and hrlb_moments,
 * bit for bit.  The call synchronises `stream` once, after uploading the tables (host
 * staging), and leaves the steps enqueued.  Every call on one GPU uses that GPU's array,
 * which keeps the last call's contents (flags and residuals are cleared at each call):
 * calls that overlap on one GPU, on different streams or threads, race.  Numerical faults
 * are not read back; a non-finite moment table shows them.
 * Errors: HRLB_EINVAL (as hrlb_init_state, nsteps < 0), HRLB_ENOMEM (state buffer too small,
 * or the batch needs more work memory than HRLB_SCRATCH_BYTES: hrlb_state_bytes' work
 * size must not exceed it), HRLB_EHIP.
 */
#define HRLB_SCRATCH_BYTES ((size_t)32 << 20)
int hrlb_step_noalloc(const hrlb_quad* q, int S, int scheme, const hrlb_params* params, int batch, void* d_state,
                      size_t state_bytes, int nsteps, double* d_moments, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HRLB_H */
