/*
 * rbe2d.h -- C ABI of librbe2d.so, an MI355X (gfx950) implementation of the
 * random batch Ewald method for charges in a doubly periodic slab with
 * dielectric jumps at its two faces (RBE2D; Gan, Gao, Liang, Xu,
 * arXiv:2405.06333, Algorithm 2).
 *
 * Physics and notation
 *   N point charges q_i at r_i = (x_i, y_i, z_i) with 0 < z_i < H, periodic
 *   in x (period Lx) and y (Ly); dielectric contrast gamma_bot at z = 0 and
 *   gamma_top at z = H (Eq. (3.1)); image series truncated at order M
 *   (Eqs. (3.2)-(3.3)): the order-l image above the slab has weight
 *   gamma_top^ceil(l/2) gamma_bot^floor(l/2) and z = (-1)^l z + 2 ceil(l/2) H,
 *   the one below gamma_bot^ceil(l/2) gamma_top^floor(l/2) and
 *   z = (-1)^l z - 2 floor(l/2) H.  Coulomb constant 1, eps_c = 1 (Eq. (2.1));
 *   every energy, force and gradient is multiplied by coulomb_prefactor.
 *
 *   Energy (Eq. (3.11)-(3.18), ELC and remainder terms dropped):
 *     E = E_real + E_k + E_self + E_ibc
 *     E_real  erfc real-space sum over real charges and images with d < r_c
 *             (Eq. (3.12); minimum image in x, y; hard cutoff)
 *     E_k     random batch estimator of the first term of Eq. (3.16):
 *             sum_l c_l Re(rho(k_l) conj(rho^M(k_l))), c_l = 2 pi S/(V P |k_l|^2),
 *             rho(k) = sum_j q_j e^{i k.r_j}, rho^M = (1 + Y_even) rho + Y_odd rhohat
 *             (Sec. 3.4), k_l = 2 pi (nx/Lx, ny/Ly, nz/Lz_ext)
 *     E_self  -alpha/sqrt(pi) sum_i q_i^2
 *     E_ibc   U_IBC^M of Theorem 3.3
 *   Forces are -grad E at fixed k-set (k-space: Eq. (3.25)-(3.26)).
 *   V = Lx Ly Lz_ext, S = sum_{k != 0} exp(-k^2/4 alpha^2) (Eq. (2.21)).
 *
 * Conventions
 *   - Every function returns rbe2d_status (0 = OK, < 0 = error) and never
 *     aborts or exits.  A message for the last error of a handle is returned
 *     by rbe2d_last_error.
 *   - Arrays marked "device" are device pointers (hipMalloc / torch CUDA
 *     tensors) owned by the caller, FP64, contiguous: positions and forces
 *     are N x 3 row-major (x, y, z per particle).  The handle owns its
 *     workspaces; they are sized at create time from n_max and nothing is
 *     allocated afterwards.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Compute calls only enqueue work on it and never synchronise, so they
 *     can be captured into a hipGraph; only rbe2d_check and rbe2d_get_kset
 *     synchronise.
 *   - x and y may take any value (they are wrapped); z must lie in (0, H).
 *     A z outside that range sets a device error word that the next
 *     rbe2d_check reports as RBE2D_E_RANGE; the results of that call are
 *     then undefined (but the kernels stay in bounds).
 *   - A handle is not thread-safe; distinct handles are independent.
 *     Overlapping calls on one handle from different streams race.
 */
#ifndef RBE2D_H
#define RBE2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbe2d_ctx *rbe2d_handle;

typedef enum {
    RBE2D_OK = 0,
    RBE2D_E_INVAL = -1,   /* bad argument or parameter                    */
    RBE2D_E_NOMEM = -2,   /* device or host allocation failed             */
    RBE2D_E_HIP = -3,     /* a HIP runtime call failed                    */
    RBE2D_E_STATE = -4,   /* call not valid in the handle's current state */
    RBE2D_E_RANGE = -5    /* a particle was outside 0 < z < H             */
} rbe2d_status;

/* Precision of the k-space phases and transcendentals. */
enum {
    RBE2D_PREC_FP64 = 0,        /* FP64 throughout                                   */
    RBE2D_PREC_FP32_PHASE = 1   /* FP32 phases, sin/cos, erfc/exp; FP64 geometry,
                                   FP64 rho(k) accumulation across particle tiles,
                                   FP64 per-k coefficients                          */
};

/* Flags of rbe2d_forces. */
enum {
    RBE2D_KSPACE = 1,        /* random batch k-space term           */
    RBE2D_REAL = 2,          /* real-space erfc term with images     */
    RBE2D_IBC = 4,           /* IBC term (and the self energy)       */
    RBE2D_ALL = 7,
    RBE2D_ACCUMULATE = 16    /* add to F instead of overwriting it   */
};

typedef struct {
    double Lx, Ly, H;          /* box: periods in x, y and slab thickness (> 0)           */
    double Lz_ext;             /* extended periodic height; <= 0 selects the smallest
                                  value allowed by Eq. (3.23) at tolerance eps_lz        */
    double eps_lz;             /* tolerance for the automatic Lz_ext (<= 0 -> 1e-6)      */
    double gamma_top;          /* contrast at z = H, |gamma_top| <= 1                    */
    double gamma_bot;          /* contrast at z = 0, |gamma_bot| <= 1                    */
    double alpha;              /* Ewald splitting parameter (> 0)                        */
    double r_c;                /* real-space cutoff, 0 < r_c <= min(Lx, Ly)/2            */
    int32_t P;                 /* wave vectors per batch, 1 <= P <= 65536                */
    int32_t M;                 /* image order, 0 <= M <= 64                              */
    int32_t precision;         /* RBE2D_PREC_*                                           */
    int32_t reserved;          /* must be 0                                              */
    int64_t n_max;             /* largest N a call may pass (>= 0)                       */
    double coulomb_prefactor;  /* scale of all energies/forces (0 -> 1.0)                */
} rbe2d_params;

/* Validates *p, derives Lz_ext, V and S (Eq. (2.21)), uploads the image and
 * sampling tables, allocates every workspace for up to p->n_max particles on
 * the current HIP device, and returns a handle in *out.  The k-set starts
 * out undefined: set one with rbe2d_set_kset or rbe2d_sample_kset.
 * Errors: RBE2D_E_INVAL (parameters, out == NULL), RBE2D_E_NOMEM,
 * RBE2D_E_HIP.  On error *out is set to NULL. */
rbe2d_status rbe2d_create(const rbe2d_params *p, rbe2d_handle *out);

/* Frees the handle and its device memory (after synchronising the device).
 * NULL is ignored. */
void rbe2d_destroy(rbe2d_handle h);

/* Returns the derived extended height, V = Lx Ly Lz_ext and S (Eq. (2.21)).
 * Any output pointer may be NULL. */
rbe2d_status rbe2d_query(rbe2d_handle h, double *Lz_ext, double *V, double *S);

/* Pure host function.  Draws P integer vectors n != 0, i.i.d. with
 * probability proportional to exp(-|k|^2/(4 alpha^2)), k = 2 pi (nx/Lx,
 * ny/Ly, nz/Lz_ext) -- the importance distribution of Sec. 2.3, sampled
 * exactly (with replacement) instead of by a Metropolis chain.  Each axis is
 * drawn by inverse CDF over |n| <= ceil(10 sigma) + 1, sigma = alpha L /
 * (sqrt(2) pi), from a counter-based SplitMix64 stream keyed by (seed,
 * stream_id); a zero vector is redrawn (at most 64 attempts, else
 * RBE2D_E_STATE).  Writes P x 3 int32 to n_out (host).  The device sampler
 * (rbe2d_sample_kset) draws the identical vectors. */
rbe2d_status rbe2d_draw_kset(const rbe2d_params *p, uint64_t seed, uint64_t stream_id,
                             int32_t *n_out);

/* Makes n (P x 3 int32, host or device per n_is_device) the handle's k-set.
 * Entries must be nonzero vectors with |n_d| < 2^20 (FP32 phases: |n_d| <
 * 2^b, the smallest power of two above every |n| the sampler can draw for
 * the system); a host array is checked (RBE2D_E_INVAL), a device array is
 * not. */
rbe2d_status rbe2d_set_kset(rbe2d_handle h, const int32_t *n, int n_is_device, void *stream);

/* Draws the handle's k-set on the device (same vectors as rbe2d_draw_kset
 * with the same seed and stream_id).  Enqueued only; graph-capturable. */
rbe2d_status rbe2d_sample_kset(rbe2d_handle h, uint64_t seed, uint64_t stream_id, void *stream);

/* Copies the current k-set to n_host (P x 3 int32) and synchronises. */
rbe2d_status rbe2d_get_kset(rbe2d_handle h, int32_t *n_host, void *stream);

/* Forces (and optionally energies) for N <= n_max charges: the RBE2D
 * splitting of Theorem 3.3 (Eq. (3.16) with the ELC and remainder terms
 * dropped), the k-space part by the random batch estimator over the handle's
 * k-set with the recalibrated structure factors of Sec. 3.4 (force:
 * Eqs. (3.25)-(3.26)), the real-space part by the erfc pair sum of Eq. (3.12)
 * over real charges and images within r_c, plus the IBC and self terms.
 *   pos    device, N x 3      q      device, N
 *   F      device, N x 3, written (or accumulated with RBE2D_ACCUMULATE)
 *   energy device, 5 doubles or NULL: {total, real, kspace, self, ibc}
 *          (parts excluded by flags are 0; self goes with RBE2D_KSPACE)
 * N == 0 is valid (energy set to 0).  Errors: RBE2D_E_INVAL (N < 0,
 * N > n_max, NULL pointers with N > 0, bad flags), RBE2D_E_STATE (no
 * k-set), RBE2D_E_HIP (launch failure). */
rbe2d_status rbe2d_forces(rbe2d_handle h, int64_t N, const double *pos, const double *q,
                          double *F, double *energy, uint32_t flags, void *stream);

/* Energy only (Theorem 3.3: E_real of Eq. (3.12), the k-space estimator
 * sum_l c_l Re(rho(k_l) conj(rho^M(k_l))) with the weights of Eq. (3.26),
 * E_self and U_IBC^M): energy (device, 5 doubles) as in rbe2d_forces with
 * RBE2D_ALL.  Same errors. */
rbe2d_status rbe2d_energy(rbe2d_handle h, int64_t N, const double *pos, const double *q,
                          double *energy, void *stream);

/* Adjoint of rbe2d_energy (the derivatives of the energy of Theorem 3.3
 * with Eq. (3.12) and the estimator of Eqs. (3.25)-(3.26)) at the current
 * k-set: given gE = dL/dE (device
 * scalar), writes dL/dr (device N x 3), dL/dq (device N) and
 * dL/dgamma (device 2: top, bot); any output may be NULL.  Nothing of size
 * N x P is stored: when the call directly follows rbe2d_energy on the same
 * handle, pos, q and N (same pointers, contents unchanged), with no other
 * call on the handle in between, the P per-k values (rho, A, B) and the
 * per-particle real-space results that call left are reused; otherwise
 * rho(k) and the real-space sums are recomputed.  dE/dq_i = phi_i, the electrostatic potential at
 * r_i of all other charges, all images (own images included) and the
 * k-space/IBC/self terms, taken literally (no neutralising background). */
rbe2d_status rbe2d_energy_backward(rbe2d_handle h, int64_t N, const double *pos,
                                   const double *q, const double *gE, double *dEdr,
                                   double *dEdq, double *dEdgamma, void *stream);

/* n_steps velocity-Verlet steps (Algorithm 2 without thermostat) with unit
 * masses: v += dt/2 F; r += dt v; x, y wrapped; z reflected specularly at
 * z_lo and z_hi (0 < z_lo < z_hi < H); a fresh k-set drawn on the device
 * from (seed, stream_id = step0 + step); F recomputed (RBE2D_ALL);
 * v += dt/2 F.  F must hold the forces of the initial positions on entry.
 * pos, vel, F (device N x 3) are updated in place.  Enqueued only.
 * With use_graph != 0 one step is captured into a hipGraph (on a private
 * stream, the step index read from a device counter) and replayed n_steps
 * times on `stream`; the graph is kept and reused while the arrays, dt,
 * walls, seed and particle counts stay the same (capturing it creates a
 * stream and instantiates a graph: the only host-side allocations after
 * create).  Both modes give bitwise identical results. */
rbe2d_status rbe2d_md_run(rbe2d_handle h, int64_t N, double *pos, double *vel, const double *q,
                          double *F, double dt, double z_lo, double z_hi, uint64_t seed,
                          int64_t step0, int32_t n_steps, int32_t use_graph, void *stream);

/* ---------------------------------------------------------------------------
 * Batches of independent systems (replicas).  One handle holds n_sys slabs,
 * each with its own rbe2d_params (box, contrasts, alpha, r_c, M, n_max); P
 * and precision must be the same for all.  Every kernel of a call covers
 * all systems at once: the particles of system r are rows
 * offsets[r] .. offsets[r+1]-1 of the caller's arrays (offsets: host,
 * n_sys + 1 int64, offsets[0] = 0, nondecreasing, each count <= that
 * system's n_max).  The k-set of a batched handle is n_sys x P x 3 int32,
 * system-major, in rbe2d_set_kset / rbe2d_get_kset; rbe2d_sample_kset
 * draws system r from stream id (stream_id + r).  Results per system equal
 * those of a single-system handle with the same params and k-set up to
 * summation order.  The single-system calls (rbe2d_forces, rbe2d_energy,
 * rbe2d_energy_backward, rbe2d_md_run) return RBE2D_E_STATE on a batched
 * handle.
 * ------------------------------------------------------------------------- */

/* Creates a handle over n_sys (1..65536) systems; params is a host array of
 * n_sys entries.  Workspaces are sized for the sum of the n_max. */
rbe2d_status rbe2d_batch_create(int32_t n_sys, const rbe2d_params *params, rbe2d_handle *out);

/* Lz_ext, V and S of system `sys` (rbe2d_query is system 0). */
rbe2d_status rbe2d_query_system(rbe2d_handle h, int32_t sys, double *Lz_ext, double *V, double *S);

/* rbe2d_forces for all systems: pos, q, F cover offsets[n_sys] rows; energy
 * (device, 5 doubles per system, system-major) or NULL. */
rbe2d_status rbe2d_batch_forces(rbe2d_handle h, const int64_t *offsets, const double *pos,
                                const double *q, double *F, double *energy, uint32_t flags,
                                void *stream);

/* rbe2d_md_run for all systems, walls at z = wall_margin and
 * z = H_r - wall_margin of each system (0 < wall_margin < min H / 2).  Step s
 * of system r draws its k-set from stream id (step0 + s) * n_sys + r. */
rbe2d_status rbe2d_batch_md_run(rbe2d_handle h, const int64_t *offsets, double *pos, double *vel,
                                const double *q, double *F, double dt, double wall_margin,
                                uint64_t seed, int64_t step0, int32_t n_steps, int32_t use_graph,
                                void *stream);

/* ---------------------------------------------------------------------------
 * MD around the path (Sec. 3.5, Sec. 4.1): Langevin thermostat and the
 * short-range repulsion of the primitive model.  Not part of the RBE2D
 * estimator; they make thermostatted runs of charged soft spheres possible.
 *   Ion-ion: purely repulsive shifted-truncated LJ,
 *     U = 4 eps [(sigma/r)^12 - (sigma/r)^6 + 1/4] for r < 2^(1/6) sigma,
 *     real ions only (no images), minimum image in x and y.
 *   Walls: the same form in the distance h to z = 0 and to z = H with
 *     sigma_wall, eps_wall (the paper gives only these two parameters).
 *   Thermostat: the Langevin equation m dv = (F - gamma v) dt
 *     + sqrt(2 gamma kT) dW (unit masses), integrated with BAOAB
 *     (Leimkuhler and Matthews 2013): v += dt/2 F; r += dt/2 v;
 *     v = c1 v + c2 xi (c1 = exp(-gamma dt), c2 = sqrt((1 - c1^2) kT));
 *     r += dt/2 v; new forces; v += dt/2 F.  gamma = 0 is velocity Verlet.
 *     xi: standard normals from the k-sampler's SplitMix64 generator keyed by
 *     (seed, 2^63 + stream) with stream = step * n_sys + system, uniforms
 *     u1, u2 at counters 2(3i+c), 2(3i+c)+1 for particle i (index within its
 *     system) and component c, xi = sqrt(-2 ln(1-u1)) cos(2 pi u2).
 * ------------------------------------------------------------------------- */
typedef struct {
    double gamma;              /* friction rate (1/time), >= 0                         */
    double kT;                 /* thermostat temperature (energy units), >= 0          */
    double sigma, eps;         /* ion-ion WCA; eps = 0 turns it off (sigma > 0 else)   */
    double sigma_wall, eps_wall; /* wall WCA; eps_wall = 0 turns it off                */
    double wall_margin;        /* integrator reflects z at wall_margin and H - wall_margin;
                                  0 < wall_margin < H/2 of every system                */
} rbe2d_md_params;

/* Short-range forces of *mp at the given positions: ADDS the ion-ion and
 * wall forces to F (device, offsets[n_sys] x 3) and, if energy is not NULL,
 * writes {E_ion_ion, E_wall} per system (device, 2 doubles per system).
 * offsets as in rbe2d_batch_forces ({0, N} for a single system); pos, q
 * device (q fills the cell list's records).  Enqueued only.  Errors:
 * RBE2D_E_INVAL (offsets, parameters, NULL arrays). */
rbe2d_status rbe2d_short_forces(rbe2d_handle h, const int64_t *offsets, const double *pos,
                                const double *q, double *F, double *energy,
                                const rbe2d_md_params *mp, void *stream);

/* n_steps BAOAB steps of all systems: forces are the RBE2D forces
 * (RBE2D_ALL, a fresh device k-set per step from (seed, step * n_sys +
 * system)) plus the short-range forces of *mp.  F must hold the total
 * forces of the initial positions on entry (rbe2d_forces or
 * rbe2d_batch_forces, then rbe2d_short_forces).  Same graph and stream
 * semantics as rbe2d_md_run; offsets as in rbe2d_batch_forces. */
rbe2d_status rbe2d_md_run_ex(rbe2d_handle h, const int64_t *offsets, double *pos, double *vel,
                             const double *q, double *F, double dt, const rbe2d_md_params *mp,
                             uint64_t seed, int64_t step0, int32_t n_steps, int32_t use_graph,
                             void *stream);

/* ---------------------------------------------------------------------------
 * Parameter selection and the stochastic error of the k-space force.
 * ------------------------------------------------------------------------- */

/* Pure host function.  Fills, for N charges in an Lx x Ly x H slab with the
 * given contrasts and a target tolerance tol in (0, 1):
 *   alpha = (N / (Lx Ly H))^(1/3) (Sec. 2.4: independent of Lz);
 *   r_c such that exp(-alpha^2 r_c^2) = tol, at most min(Lx, Ly)/2 (then
 *     alpha = sqrt(ln(1/tol)) / r_c);
 *   M, the smallest order (<= 64) whose image truncation estimate of
 *     Theorem 3.2, |gamma_top|^floor((M+1)/2) |gamma_bot|^ceil((M+1)/2)
 *     exp(-2 pi H (M-1) / max(Lx, Ly)), is at most tol;
 *   eps_lz = tol and Lz_ext from Eq. (3.23);
 * and copies Lx, Ly, H, gamma_top, gamma_bot into *p.  P, precision, n_max,
 * reserved and coulomb_prefactor are left as they are.  Errors:
 * RBE2D_E_INVAL. */
rbe2d_status rbe2d_suggest_params(int64_t N, double Lx, double Ly, double H, double gamma_top,
                                  double gamma_bot, double tol, rbe2d_params *p);

/* Per-particle estimate of E|Xi_i|^2, the variance of the RBE k-space force
 * of particle i (Theorem 2.2), from the current k-set: the P per-k force
 * terms t_l(i) are i.i.d. given the positions and sum to F_i^k, so
 * var_i = (P sum_l |t_l(i)|^2 - |F_i^k|^2) / (P - 1) is unbiased (0 when
 * P = 1).  var: device, offsets[n_sys] doubles.  offsets as in
 * rbe2d_batch_forces ({0, N} for a single system).  Enqueued only.  Errors
 * as rbe2d_batch_forces. */
rbe2d_status rbe2d_force_variance(rbe2d_handle h, const int64_t *offsets, const double *pos,
                                  const double *q, double *var, void *stream);

/* Autotuner.  Times, with HIP events on `stream`, the candidate launch
 * parameters of the evaluation for the particle layout given by offsets
 * (host, n_sys + 1 int64, as in rbe2d_batch_forces; {0, N} for a single
 * system) on the caller's pos and q (device) and the current k-set:
 * particles per thread of the structure-factor tiles (1..16), the k-range
 * split of the force pass (1..64) and, for small systems, the x-column split
 * of the pair work (1..5).  The fastest are kept in the handle and used by
 * every later call with the same per-system counts (other layouts use the
 * built-in heuristics); a cached MD graph is dropped.  Writes the three
 * choices to chosen (host int[3]) when not NULL.  Synchronises `stream`;
 * not to be called during graph capture.  Results of later calls change only
 * by summation order.  Errors as rbe2d_batch_forces. */
rbe2d_status rbe2d_autotune(rbe2d_handle h, const int64_t *offsets, const double *pos, const double *q,
                            int32_t *chosen, void *stream);

/* Kernel timing (tracing).  rbe2d_profile_enable(h, n) creates n event
 * pairs per kernel class and from then on brackets every launch of each
 * class with HIP events on the launch stream (n = 0 turns timing off and
 * frees the events).  rbe2d_profile_read synchronises the device and
 * writes, for each of the first n_slots classes, the summed duration in
 * milliseconds and the number of launches timed since the last read (a
 * class launched more than n times between reads keeps its first n).
 * Classes: 0 prep, 1 structure-factor pass, 2 per-k reduce/assemble,
 * 3 cell-list build, 4 real-space pairs, 5 force scatter, 6 energies,
 * 7 integrator, 8 k-sampler, 9 short-range forces, 10 real-space add (and
 * the fused closing half kick of MD steps).  Not to be used while a graph is
 * captured. */
enum { RBE2D_PROF_SLOTS = 11 };
rbe2d_status rbe2d_profile_enable(rbe2d_handle h, int32_t n_events);
rbe2d_status rbe2d_profile_read(rbe2d_handle h, double *ms, int64_t *launches, int32_t n_slots);

/* Restricts the timing to the classes whose bit is set in class_mask (bit
 * i = class i above); rbe2d_profile_enable selects all classes.  Each timed
 * launch adds two event records to its stream, so timing one class perturbs
 * the timed work least.  Errors: RBE2D_E_INVAL (NULL handle). */
rbe2d_status rbe2d_profile_classes(rbe2d_handle h, uint32_t class_mask);

/* Surface charge densities on the interfaces (the remark after Eq. (3.26);
 * its formula is in a supplement that is not available, so the terms are
 * derived here from the image series of Sec. 3.1 and Theorem 3.3):
 * sigma_bot on z = 0 and sigma_top on z = H, for system `sys` of the handle
 * (-1: every system).  They are uniform sheets just inside the slab whose
 * images follow the image series; with the sheets the ions are in general
 * not neutral, and the k-space reformulation then needs the net-charge term
 * of its k_x = k_y = 0 modes.  Both additions belong to the IBC part
 * (RBE2D_IBC, energy component 4):
 *   sheets      E = sum_i q_i phi_s(z_i), phi_s(z) = -2 pi sum_{sheets, images}
 *               w sigma |z - z_w| (uniform field in the slab);
 *   net charge  U_Q = -(pi / V) sum_{i, j, images w} q_i q_j w (z_i^2 + z_j^w^2).
 * Position-independent terms are dropped: with a net ionic charge the
 * energy is defined up to a constant (forces are unique).  sigma_top =
 * sigma_bot = 0 (the state after create) turns both off.  Synchronises the
 * device; not to be called during graph capture.  Errors: RBE2D_E_INVAL. */
rbe2d_status rbe2d_set_surface_charges(rbe2d_handle h, int32_t sys, double sigma_top, double sigma_bot);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rbe2d_forces without a
 * handle.  Every workspace lives in one 32 MiB file-scope device array of
 * the library (each GPU that runs this call holds its own copy until the
 * process ends); the call allocates no device or pinned memory, creates no
 * stream or event and only enqueues kernels on `stream`, so it can be
 * captured.  Host-side set-up work (the derived constants and tables of *p)
 * is redone only when *p changes between calls.
 *   p        parameters as for rbe2d_create; n_max <= 32768 and P <= 1024
 *            (larger values return RBE2D_E_INVAL with a message)
 *   kset     device, P x 3 int32, the k-set (not checked; see rbe2d_set_kset)
 *   N, pos, q, F, energy, flags   as in rbe2d_forces (N <= p->n_max)
 *   err_word device int32 or NULL: receives the device error word of this
 *            call (bit 0: a z outside (0, H), as RBE2D_E_RANGE of rbe2d_check)
 * Results equal rbe2d_forces on a handle with the same parameters and k-set
 * up to summation order.  Calls on one GPU share its array, which keeps the
 * last call's contents (each call rewrites everything it reads): calls that
 * overlap on one GPU (other streams, other threads) race.  Errors:
 * RBE2D_E_INVAL (arguments, sizes beyond the maximum), RBE2D_E_HIP; the
 * message is rbe2d_last_error(NULL). */
rbe2d_status rbe2d_forces_noalloc(const rbe2d_params *p, const int32_t *kset, int64_t N, const double *pos,
                                  const double *q, double *F, double *energy, uint32_t flags,
                                  int32_t *err_word, void *stream);

/* Synchronises `stream` and reports asynchronous errors: RBE2D_E_RANGE if a
 * call since the last check saw z outside (0, H), RBE2D_E_HIP for a failed
 * kernel.  Clears the device error word. */
rbe2d_status rbe2d_check(rbe2d_handle h, void *stream);

/* Message of the handle's last error ("" if none).  With h == NULL, the
 * message of the last failed rbe2d_create in this thread. */
const char *rbe2d_last_error(rbe2d_handle h);

#ifdef __cplusplus
}
#endif
#endif /* RBE2D_H */
