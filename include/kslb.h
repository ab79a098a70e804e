/*
 * kslb.h -- C ABI of the MI355X (gfx950) lattice Boltzmann solver for the
 * Kuramoto-Sivashinsky equation, after Otomo, Boghosian and Dubois,
 * "Efficient lattice Boltzmann models for the Kuramoto-Sivashinsky equation"
 * (arXiv:1711.03540).
 *
 * The method (paper section 2): populations f_i on a periodic 1D lattice with
 * velocities c_i in {0, +-1, +-2} (D1Q5, "basic scheme") or {0, +-1, +-2, +-3}
 * (D1Q7, "improved scheme") follow the BGK lattice Boltzmann equation, Eq. (2),
 *     f_i(x + c_i, t + 1) - f_i(x, t) = -(f_i - feq_i) / tau,
 * with rho = sum_i f_i and the equilibrium of Eq. (3) / section 2.3,
 *     feq_i = rho (w0_i + K w2_i + M' w4_i + C6 w6_i) + rho^2 J w1_i,
 * where J, K, M come from Table 2, M' = M + dM (Eq. (delta_M)) and C6 (the
 * delta f_eq correction of section 2.2) are used by D1Q7 only, and the
 * weights are those of appendix A.  Physical space and time are X = dX x and
 * T = dT t (Eq. (scaling)).  All of this folds into two per-velocity vectors,
 *     feq_i(rho) = E_i rho + G_i rho^2,
 * with G_i = J w1_i nonzero only for c_i = +-1, +-2.
 *
 * Conventions that hold for every entry point:
 *   - Velocity order i = 0..Q-1 is c = (0, +1, -1, +2, -2[, +3, -3]).
 *   - Site j sits at X_j = j dX; the lattice is periodic with n_sites sites.
 *   - Population arrays exchanged with the caller are Q x n_sites doubles,
 *     population-major (element (i, j) at index i * n_sites + j).
 *   - The stored state is the post-collision one; the density after n steps
 *     is rho_j = sum_i f_i(j) of the paper's f at time n.
 *   - Device memory and HIP streams belong to the caller.  The library never
 *     frees a caller buffer.  It allocates only small descriptor tables, the
 *     exchange area of the SPAN kernel (for each exchange of one launch, one
 *     copy of every workgroup's own sites; at most 256 MiB, a longer advance
 *     being split into several launches) and, when a host pointer is passed
 *     to a transfer call, one device staging buffer of Q * n_sites doubles;
 *     all live until destroy.  The SPAN kernel's control words (abort word,
 *     sticky error word, count of aborted launches) sit in the diagnostics
 *     area of the lattice's own buffer.
 *   - Every function returns a kslb_status (0 = OK, < 0 = error) and never
 *     aborts or throws; kslb_last_error() describes the last failure of the
 *     calling thread.  Work enqueued on the stream is asynchronous; a device
 *     fault surfaces at the next synchronising call.
 *   - An object is not thread-safe; distinct objects are independent and may
 *     be used from different threads at once (the library's process-wide
 *     caches, per-kernel LDS limits and device occupancy, are locked).
 *   - A SPAN launch whose wait for a neighbour's edge times out (or that is
 *     aborted) stops early without writing its result.  From then until the
 *     state is replaced (kslb_init_rho, kslb_write_f, kslb_load_state) the
 *     lattice's sticky error word is set: later SPAN launches return at
 *     once, readouts into device memory write NaN, and readouts into host
 *     memory, kslb_save_state and kslb_diagnostics return KSLB_EDEVICE.
 *     kslb_aborted_launches counts such launches over the lattice's life.
 *   - Failure-path testing: with the environment variable
 *     KSLB_SPAN_INJECT_ABORT=1, every SPAN launch starts with its abort word
 *     raised; it stops at its first edge exchange, as after a timed-out wait.
 */
#ifndef KSLB_H
#define KSLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kslb_lattice kslb_lattice;
typedef struct kslb_ensemble kslb_ensemble;

typedef enum {
    KSLB_OK = 0,
    KSLB_EINVAL = -1,      /* bad argument or shape */
    KSLB_ENOMEM = -2,      /* buffer too small or allocation failed */
    KSLB_EDEVICE = -3,     /* HIP runtime error */
    KSLB_ESTATE = -4,      /* call out of order (e.g. advance before init) */
    KSLB_EUNSTABLE = -5,   /* the linear stability guard refused the parameters */
    KSLB_ENONFINITE = -6   /* a non-finite value was found in the state */
} kslb_status;

enum { KSLB_D1Q5 = 5, KSLB_D1Q7 = 7 };

/* Storage precision of the populations.
 *   FP64  : f_i stored and updated in double precision.
 *   FP32  : f_i stored in single precision; the density sum and the rho^2
 *           term of the equilibrium in double, the relaxation in single.
 *   SPLIT : rho stored in double and the non-equilibrium part
 *           f_i - feq_i(rho) in single; arithmetic in double.  Exact change
 *           of variables of the FP64 scheme (rounding aside).
 *   RHO   : tau = 1 only.  With omega = 1 the collision of Eq. (2) leaves
 *           f_i = feq_i(rho), so the state is rho alone (one double per
 *           site); densities are bitwise those of FP64 at tau = 1.  Setting
 *           any other tau returns EINVAL.                                  */
enum { KSLB_FP64 = 0, KSLB_FP32 = 1, KSLB_SPLIT = 2, KSLB_RHO = 3 };

/* Reading of the bracket of Eq. (delta_M).  DERIVED uses (T3+1)/(T2+1), the
 * ratio in the fourth-derivative term of Eq. (KS_trunc2) that dM cancels;
 * LITERAL uses (T3+1)/(T4+1) as printed.  They coincide at tau = 1.        */
enum { KSLB_DM_DERIVED = 0, KSLB_DM_LITERAL = 1 };

/* Linear stability guard (see kslb_stability_check). */
enum { KSLB_GUARD_REFUSE = 0, KSLB_GUARD_RAISE_TAU = 1, KSLB_GUARD_OFF = 2 };

/* Kernel class used by kslb_advance.
 *   AUTO     : the library's choice: SPAN for lattices of up to 65536 sites
 *              that it can split, else RESIDENT when the lattice fits one
 *              workgroup's registers, else TILED.
 *   PLAIN    : one fused stream+collide step per launch (HBM ping-pong).
 *   RESIDENT : one workgroup holds the whole lattice in registers for all
 *              steps; needs n_sites = B * L with B in {4, 8}, L <= 512.
 *   TILED    : halo-widened tiles, several steps per launch in registers:
 *              windows of 256 lanes x B sites (B = 12 for FP64, 10 for FP32,
 *              8 for split, 32 for the rho-only state) each keep
 *              W - 2 max|c| s sites after s steps (by default 80 for D1Q7
 *              FP64, 112 for D1Q5 FP64, 48 for FP32, 32 for D1Q7 and 40
 *              for D1Q5 split, 64 for the rho-only D1Q7 state, 128 for the
 *              rho-only D1Q5 state).
 *   SPAN     : thousands of steps per launch; single-wave workgroups each
 *              hold W = 64 B sites in registers (B = 2 sites per lane for
 *              the population states, max|c| for the rho-only state): their
 *              own W - 2 max|c| s sites and a halo of max|c| s sites per
 *              side, refreshed every s steps from the own sites the other
 *              workgroups publish in a library-owned exchange area (a halo
 *              may reach past the nearest neighbour).  s is the
 *              steps_per_launch of kslb_set_kernel; by default the largest
 *              with 3 W >= 8 max|c| s whose owners fit (16 for D1Q7 and 24
 *              for D1Q5 population states, 24 for the rho-only state).  Every owner
 *              waits on its neighbours, so all must be resident at once: a
 *              plan uses at least 2 and at most half of the owners the
 *              device keeps resident (its occupancy for the kernel times
 *              its compute units; 1024 on MI355X), leaving the rest for
 *              other work.  SPAN lattices advanced at the same time on
 *              other streams, or other work holding every compute unit,
 *              can still starve a launch; its waits are bounded and it then
 *              stops with the error described above.
 * All classes give bitwise identical results.                              */
enum { KSLB_KERNEL_AUTO = 0, KSLB_KERNEL_PLAIN = 1, KSLB_KERNEL_RESIDENT = 2,
       KSLB_KERNEL_TILED = 3, KSLB_KERNEL_SPAN = 4 };

/* ---------------------------------------------------------------------- */
/* Host-only parameter functions (no device work).                         */
/* ---------------------------------------------------------------------- */

/* Coefficients of the scheme for q in {5, 7}, alpha = dX > 0, beta = dT > 0,
 * tau >= 0.92 (M has a pole where T4 + 1 = 0, near tau = 0.908).
 * jkm[5] receives {J, K, M, dM, C6} (Table 2; Eq. (delta_M); section 2.2;
 * dM = C6 = 0 for D1Q5).  E[q], G[q] (either may be NULL) receive the folded
 * equilibrium vectors, feq_i = E_i rho + G_i rho^2.                         */
kslb_status kslb_scheme_coefficients(int q, double dX, double dT, double tau, int dm_variant,
                                     double* jkm, double* E, double* G);

/* The paper's fitted minimum stable tau, Eq. (general_tau_formula) with
 * Eqs. (A_B_fit_D1Q5)/(A_B_fit_D1Q7).  Returns NaN for a bad q or dX <= 0. */
double kslb_tau_fit(int q, double dX, double dT);

/* Spectral radius of the linearised one-step operator about a uniform
 * density rho_bar, at lattice wavenumber k (radians per site):
 *     A(k) = diag(exp(-i k c)) [(1 - omega) I + omega (E + 2 rho_bar G) 1^T].
 * Host-only.                                                               */
kslb_status kslb_spectral_radius(int q, const double* E, const double* G, double omega,
                                 double rho_bar, double k, double* radius);

/* Linear stability guard.  For rho_bar in {0, +rho_max, -rho_max} and 801
 * wavenumbers k in [0, pi]: radius <= 1 + 1e-13 where k > 1.5 dX (kappa =
 * k/dX > 1.5, where the KS equation damps), radius <= exp(0.3 dT) elsewhere
 * (the KS growth rate kappa^2 - kappa^4 never exceeds 1/4).  *stable = 1 if
 * every check passes.  The paper gives no criterion for its minimum stable
 * tau (section 3); this is the library's own.                              */
kslb_status kslb_stability_check(int q, const double* E, const double* G, double omega,
                                 double dX, double dT, double rho_max, int* stable);

/* ---------------------------------------------------------------------- */
/* One lattice.                                                            */
/* ---------------------------------------------------------------------- */

/* Bytes of the caller-owned device buffer a lattice needs: two copies of the
 * state (ping-pong), each rounded up to 256 bytes, plus 4096 bytes of
 * diagnostics.  0 for bad arguments.                                        */
size_t kslb_state_bytes(int64_t n_sites, int q, int precision);

/* Create a lattice over the caller's device buffer dev_buf (>= the bytes
 * above, 256-byte aligned) on the caller's stream (a hipStream_t; NULL =
 * the null stream).  The device current at this call is the lattice's.   */
kslb_status kslb_create(kslb_lattice** out, int64_t n_sites, int q, int precision,
                        void* dev_buf, size_t buf_bytes, void* hip_stream);

/* Set alpha = dX, beta = dT and tau (tau <= 0: the paper's fitted tau),
 * computing the coefficients and omega = 1/tau, then apply the stability
 * guard at rho_max (>= 0) under guard_policy.  RAISE_TAU raises tau in steps
 * of 0.02 (at most 200 steps) until the guard passes.                      */
kslb_status kslb_set_physical(kslb_lattice* lat, double dX, double dT, double tau,
                              int dm_variant, int guard_policy, double rho_max);

/* Raw override: E[q], G[q] and omega in (0, 2).  G_i must be 0 for c_i in
 * {0, +-3}, and E must be even and G odd in c exactly (E at +c equals E at
 * -c, G at +c equals minus G at -c), the symmetry of Eq. (feq)'s weights,
 * which the kernels use; EINVAL otherwise.  No guard.                      */
kslb_status kslb_set_coefficients(kslb_lattice* lat, const double* E, const double* G,
                                  double omega);

/* Current coefficients; any output may be NULL.  jkm as in
 * kslb_scheme_coefficients (zeros after a raw override).                   */
kslb_status kslb_get_coefficients(const kslb_lattice* lat, double* E, double* G, double* omega,
                                  double* tau, double* jkm);

/* Choose the kernel class and, for TILED, the steps per launch (for SPAN,
 * the steps between edge exchanges); 0 = the library's default.  Requests
 * that the shape cannot use return EINVAL.                                 */
kslb_status kslb_set_kernel(kslb_lattice* lat, int kernel, int steps_per_launch);

/* The kernel an advance runs now, with AUTO resolved for this shape and
 * boundary: its class, the most steps one launch advances (1 for PLAIN, the
 * tile's steps for TILED, 2^20 for RESIDENT, as many as the exchange area
 * holds for SPAN; longer advances are split into launches of at most that
 * many steps), the steps between edge exchanges (SPAN; 0 otherwise), the
 * workgroups of one launch and the lanes of each.  Any output may be NULL.  Host only; enqueues nothing.
 * Every class runs the same step, Eq. (2); the class changes how steps are
 * scheduled, not what they compute.                                        */
kslb_status kslb_get_kernel(const kslb_lattice* lat, int* kernel, int* steps_per_launch,
                            int* exchange_steps, int64_t* workgroups, int* lanes_per_workgroup);

/* The kernel class and launch shape kslb_get_kernel would report for a
 * lattice of this shape, boundary (KSLB_PERIODIC / KSLB_FIXED_ENDS) and
 * kslb_set_kernel request, on a device that keeps span_owners SPAN
 * workgroups resident (a plan uses at most half) and gives one workgroup
 * lds_bytes of LDS; 0 for either queries the current device.  Host only:
 * the planning step of kslb_advance, exposed so that it can be checked
 * without a device.  EINVAL when an explicit request cannot be met.       */
kslb_status kslb_plan_kernel(int64_t n_sites, int q, int precision, int boundary, int kernel, int steps_per_launch,
                             int64_t span_owners, int lds_bytes, int* kernel_out, int* steps_per_launch_out,
                             int* exchange_steps, int64_t* workgroups, int* lanes_per_workgroup);

/* Boundary of the lattice.  KSLB_PERIODIC (default) or KSLB_FIXED_ENDS: the
 * problem of the paper's Table 3, sites 0 and n_sites-1 held at the
 * equilibrium of rho_left / rho_right, and a population streamed from beyond
 * an end taking that end's equilibrium value (the ends and max|c| ghost
 * sites beyond them are reset after every streaming; the paper gives only
 * the end values).  Fixed ends run on the PLAIN and SPAN kernels.  Set it
 * before kslb_init_rho, which then also imposes the end states.           */
enum { KSLB_PERIODIC = 0, KSLB_FIXED_ENDS = 1 };
kslb_status kslb_set_boundary(kslb_lattice* lat, int mode, double rho_left, double rho_right);

/* f := feq(rho) at every site (Eq. (feq); the paper does not state the
 * initial populations, and the equilibrium of the initial density is the
 * reading taken), step counter := 0.  rho: n_sites doubles on the device
 * (rho_on_device = 1) or the host.  Host input synchronises.               */
kslb_status kslb_init_rho(kslb_lattice* lat, const double* rho, int rho_on_device);

/* Enqueue n_steps >= 0 steps of Eq. (2) on the stream (asynchronous).      */
kslb_status kslb_advance(kslb_lattice* lat, int64_t n_steps);

/* One whole solve, enqueued on the stream: the result of kslb_init_rho(rho0,
 * on device), kslb_advance(n_steps) and kslb_read_rho(rho_out, on device),
 * bitwise, state and step count included.  rho0 and rho_out: n_sites
 * doubles of device memory owned by the caller; they may be the same
 * buffer.  On the TILED kernel with both pointers 16-byte aligned the
 * initialisation is fused into the first launch (the equilibrium of Eq.
 * (feq) formed from rho0 on load) and the readout into the last (the
 * density of section 2, sum_i f_i), except where a single launch would read
 * rho0 and write an overlapping rho_out: then the readout follows it.
 * Otherwise the three calls run as they are.  On an error from the first
 * launch the lattice holds no state (kslb_init_rho or kslb_write_f again). */
kslb_status kslb_solve(kslb_lattice* lat, const double* rho0, int64_t n_steps, double* rho_out);

/* As kslb_advance, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * it allocates nothing, host or device.  The one kernel class that needs
 * scratch, SPAN, takes its edge slots from a static 64 MiB device array the
 * library holds on each GPU until the process ends (its address is looked up
 * on a device's first call) instead of the lattice's exchange area; a longer
 * advance is split into more launches, with bitwise the same result.  Every
 * call on one GPU shares that array, which keeps the last call's contents
 * (each launch refills the slots it uses first): calls whose work overlaps on
 * one GPU (different streams, not ordered by the caller) race.  ENOMEM when
 * one exchange of the lattice's SPAN plan needs more than 64 MiB (no
 * lattice AUTO plans on SPAN does).                                        */
kslb_status kslb_advance_noalloc(kslb_lattice* lat, int64_t n_steps);

/* rho_j = sum_i f_i(j), the density of section 2 (collision conserves it,
 * so the stored post-collision state gives the same rho), into n_sites
 * doubles (device or host).  Host output synchronises the stream; device
 * output is enqueued.                                                      */
kslb_status kslb_read_rho(kslb_lattice* lat, double* out, int out_on_device);

/* Populations as Q x n_sites doubles.  pre_collision = 0: the stored state
 * after step n, i.e. the collided populations of Eq. (2)'s right-hand side
 * at time n.  pre_collision = 1: those populations streamed one lattice
 * link, S_i(j - c_i), which are the paper's not-yet-collided f_i(x_j) at
 * time n + 1 (the left-hand side of Eq. (2)).  The pre-collision f at time
 * n itself is not kept (at tau = 1 it cannot be recovered from the state). */
kslb_status kslb_read_f(kslb_lattice* lat, double* out, int out_on_device, int pre_collision);

/* Replace the state by Q x n_sites post-collision doubles and set the step
 * counter.  In FP32/SPLIT the values are rounded to the storage format.     */
kslb_status kslb_write_f(kslb_lattice* lat, const double* in, int in_on_device, int64_t step);

/* Raw state copy for bitwise checkpoints: state_size bytes (see
 * kslb_state_size) copied device-to-device on the stream, into / from a
 * caller-owned device buffer.  load_state also sets the step counter and
 * clears the error word of the multi-workgroup kernel.                     */
size_t kslb_state_size(const kslb_lattice* lat);
kslb_status kslb_save_state(kslb_lattice* lat, void* dev_dst);
kslb_status kslb_load_state(kslb_lattice* lat, const void* dev_src, int64_t step);

/* Steps advanced since the state was set (init, write_f or load_state).  */
kslb_status kslb_step_count(const kslb_lattice* lat, int64_t* step);

/* Diagnostics (synchronises): mass = sum_j rho_j in double, accumulated in a
 * fixed order; *nonfinite = 1 if any stored value is NaN or infinite.
 * KSLB_EDEVICE (after filling both) while the sticky error word is set.    */
kslb_status kslb_diagnostics(kslb_lattice* lat, double* mass, int* nonfinite);

/* SPAN launches of this lattice that stopped early (a timed-out or aborted
 * edge exchange) since it was created; replacing the state does not reset
 * it.  Synchronises.                                                       */
kslb_status kslb_aborted_launches(kslb_lattice* lat, int64_t* count);

/* Releases the library's own buffers (staging, exchange area), after
 * synchronising the stream when it holds any; never the caller's buffer.   */
kslb_status kslb_destroy(kslb_lattice* lat);

/* ---------------------------------------------------------------------- */
/* Ensembles: many independent periodic lattices, each with its own size,  */
/* scheme, storage mode, coefficients and step budget, advanced together:  */
/* each chunk of steps is one launch per (scheme, storage) present, whose  */
/* workgroups each hold tiles of one or more instances of one coefficient  */
/* set.  The one-step arithmetic of an instance is that of a lattice of the */
/* same scheme, storage and coefficients (bitwise).                        */
/* ---------------------------------------------------------------------- */

/* Device bytes for instances i = 0 .. count-1 of n_sites[i] sites, scheme
 * q[i] (KSLB_D1Q5 / KSLB_D1Q7) and storage precision[i] (host arrays): the
 * ping-pong state of each, 256-byte aligned, plus diagnostics.  0 for a bad
 * shape.                                                                   */
size_t kslb_ensemble_bytes(int count, const int64_t* n_sites, const int* q, const int* precision);

/* Carve the caller's device buffer (>= kslb_ensemble_bytes, 256-byte
 * aligned; never freed by the library) into the instances' states; work is
 * enqueued on the caller's stream.  The arrays are copied.                 */
kslb_status kslb_ensemble_create(kslb_ensemble** out, int count, const int64_t* n_sites, const int* q,
                                 const int* precision, void* dev_buf, size_t buf_bytes, void* hip_stream);

/* Coefficients of instance idx, or of every instance for idx = -1 (one set
 * per scheme present), as kslb_set_physical: dX, dT, tau <= 0 for the fit of
 * Eq. (general_tau_formula), the delta-M reading, the stability guard and
 * its rho_max.  For idx = -1 nothing is assigned unless every instance's
 * set is valid.  KSLB_RHO instances need tau = 1.  An instance's state is
 * kept: new coefficients apply from its next step.                         */
kslb_status kslb_ensemble_set_physical(kslb_ensemble* ens, int idx, double dX, double dT, double tau,
                                       int dm_variant, int guard_policy, double rho_max);

/* Tiling knobs (0 keeps the current value):
 *   sites_per_lane  4 or 8 (window of 256 lanes x that many sites; 10 when
 *                   every instance has FP32 storage, 12 when every instance
 *                   has FP64 storage, 16 when every instance has the rho-only
 *                   storage); EINVAL otherwise;
 *   max_segments    instance tiles one workgroup window may hold, 1..256
 *                   (1 = one tile per workgroup);
 *   steps_per_chunk steps per launch, with 2 max|c| steps < the window.
 * Defaults: 8 sites (12 when every instance has FP64 storage, 10 when every
 * instance has FP32 storage), 16 segments, 64 steps (48 when every instance
 * has FP32 storage, 40 when any has split storage).                        */
kslb_status kslb_ensemble_set_tiling(kslb_ensemble* ens, int sites_per_lane, int max_segments,
                                     int steps_per_chunk);

/* The tiling in effect (any output pointer may be NULL).  Host only.      */
kslb_status kslb_ensemble_get_tiling(const kslb_ensemble* ens, int* sites_per_lane, int* max_segments,
                                     int* steps_per_chunk);

/* Steady-state graphs (default on): when every instance still to advance
 * has at least four more full chunks, the two alternating chunk launches are
 * captured as a HIP graph (kernel nodes only) and replayed, provided one call
 * replays them at least four times or the same pair recurs from the
 * previous call; otherwise they are launched directly.  A replaced graph is
 * destroyed once its replays have completed, without blocking the caller.
 * Results are bitwise those of the launch-per-chunk path.                  */
kslb_status kslb_ensemble_set_graphs(kslb_ensemble* ens, int enable);

/* The tau instance idx uses (after the fit and the guard). */
kslb_status kslb_ensemble_get_tau(const kslb_ensemble* ens, int idx, double* tau);

/* Reuse instance idx's memory for a lattice of n_sites <= its capacity (the
 * size given at create).  Its state is dropped; init it again.             */
kslb_status kslb_ensemble_resize(kslb_ensemble* ens, int idx, int64_t n_sites);

/* Device bytes of one instance's state outside an ensemble's buffer: two
 * copies, each rounded up to 256 bytes (no diagnostics).  0 for a bad shape. */
size_t kslb_instance_bytes(int64_t n_sites, int q, int precision);

/* Rebind instance idx to a lattice of n_sites sites (its scheme and storage
 * unchanged) whose state lives in caller-owned device memory dev_state
 * (>= kslb_instance_bytes bytes, 256-byte aligned, on the ensemble's device;
 * never freed by the library).  Its capacity becomes n_sites, its state is
 * dropped (init it again) and its coefficients are kept.  Work already
 * enqueued still uses the previous memory (stream order), so the caller may
 * release that memory once such work has completed.  This lets a server size
 * each admitted request's state to the request and admit requests by a
 * device-memory budget.                                                    */
kslb_status kslb_ensemble_bind(kslb_ensemble* ens, int idx, int64_t n_sites, void* dev_state, size_t bytes);

/* As kslb_init_rho for instance idx: f := feq(rho) from its current number
 * of densities (device or host), step counter := 0.                        */
kslb_status kslb_ensemble_init_rho(kslb_ensemble* ens, int idx, const double* rho, int on_device);

/* Initialise every instance at once, as kslb_ensemble_init_rho for each:
 * rho holds the densities of all instances back to back in instance order
 * (sum over i of the current n_sites of instance i doubles), on the device
 * (on_device = 1) or the host (then the call synchronises).  One launch per
 * (scheme, storage) present instead of one per instance.  ESTATE unless
 * every instance has its coefficients.                                     */
kslb_status kslb_ensemble_init_rho_all(kslb_ensemble* ens, const double* rho, int on_device);

/* Advance instance i by steps[i] >= 0 steps (asynchronous).  Launches one
 * kernel per chunk; instances with fewer steps left drop out of later
 * chunks.                                                                  */
kslb_status kslb_ensemble_advance(kslb_ensemble* ens, const int64_t* steps);

/* As kslb_read_rho for instance idx (its current number of sites).      */
kslb_status kslb_ensemble_read_rho(kslb_ensemble* ens, int idx, double* out, int on_device);

/* The densities of every instance back to back in instance order (sum over
 * i of the current n_sites of instance i doubles), into device memory
 * (on_device = 1, enqueued) or host memory (synchronises).  One launch per
 * (scheme, storage) present.  ESTATE unless every instance has a state.    */
kslb_status kslb_ensemble_read_rho_all(kslb_ensemble* ens, double* out, int on_device);

/* Benettin renormalisation of trajectory pairs, a tool for the largest
 * Lyapunov exponent of the scheme's dynamics (the chaotic dynamics the paper
 * names as its next subject, section 4).  For each pair p of instances
 * (ref[p], pert[p]: host arrays of indices of FP64 instances of one scheme
 * with equal sites and steps; no instance perturbed twice, or both
 * reference and perturbed): with d = || S_pert - S_ref ||_2 over all Q x n stored
 * (post-collision) populations, set S_pert <- S_ref + (S_pert - S_ref) delta / d
 * and add ln(d / delta) to log_accum[p] (device array of npairs doubles, owned
 * by the caller, which zeroes it first).  A zero or non-finite d leaves the
 * pair unchanged and stores NaN in log_accum[p].  Enqueued on the ensemble's
 * stream.  EINVAL for other storage modes or bad pairs.                 */
kslb_status kslb_ensemble_renormalize(kslb_ensemble* ens, int npairs, const int* ref, const int* pert,
                                      double delta, double* log_accum);

/* Lyapunov spectrum of the scheme's dynamics (the chaotic dynamics section 4
 * names as the next subject): renormalisation of ngroups groups, each a reference
 * trajectory ref[g] and k perturbed copies pert[g k + m], m = 0..k-1
 * (1 <= k <= 8; host arrays of FP64 instances of one scheme with equal
 * sites and steps, no instance used twice).  With v_m = S_pert[m] - S_ref
 * over the Q x n stored populations, V = U R (U orthonormal, R upper
 * triangular with positive diagonal, from the Cholesky factor of the Gram
 * matrix of the v_m), S_pert[m] <- S_ref + delta u_m and
 * log_accum[g k + m] += ln(R_mm / delta) (device array of ngroups k doubles,
 * owned by the caller, which zeroes it first).  The time averages of these
 * sums are the k leading Lyapunov exponents (Benettin et al. 1980, with a QR
 * step in place of Gram-Schmidt).  A group whose R is not positive definite
 * is left unchanged and gets NaN.  Enqueued on the ensemble's stream.      */
kslb_status kslb_ensemble_orthonormalize(kslb_ensemble* ens, int ngroups, int k, const int* ref, const int* pert,
                                         double delta, double* log_accum);

/* Step counter and non-finite flag of instance idx (synchronises). */
kslb_status kslb_ensemble_status(kslb_ensemble* ens, int idx, int64_t* step, int* nonfinite);

kslb_status kslb_ensemble_destroy(kslb_ensemble* ens);

/* Thread-local description of the last failing call ("" if none). */
const char* kslb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KSLB_H */
