/*
 * reann.h -- C ABI of the MI355X (gfx950) REANN message-passing energy/force library.
 *
 * The library evaluates the REANN potential of Xia & Jiang, "Efficient
 * Parallelization of Message Passing Neural Networks":
 *   Sec. 2.1, Eq. (1)   embedded atom densities rho_i from orbital sums over the
 *                       neighbours inside r_c, squared with the l!/(lx!ly!lz!) weights;
 *   Sec. 2.1, Eq. (2)   message update c_i^t = M^{t-1}_{s_i}(rho_i^{t-1}), 1 <= t <= T-1;
 *   Sec. 2.1            atomic energies from the last atomic NN, E = sum_i E_i;
 *   Sec. 2.2            one neighbour list (cutoff r_c + skin) reused by every layer;
 *                       spatial subdomains whose ghost atoms receive their owners'
 *                       messages once per layer, emulated inside one GPU;
 *   Sec. 2.2, Eqs. (3)-(5)  forces by the chain rule, with the ghost atoms' message
 *                       adjoints (vector-Jacobian products) and forces reduced onto
 *                       their owners.
 * The problem statement (positions, species, periodic cell, r_c, T and weights in;
 * energy, forces and virial out) follows the paper's setting of periodic MD boxes
 * decomposed into subdomains (Sec. 2.2).
 *
 * Conventions for every call:
 *  - Units: Angstrom, eV, eV/Angstrom, fs.  Positions are Cartesian, FP64, [n][3] row-major.
 *  - cell[9] holds the three lattice vectors as rows; only orthorhombic cells are
 *    supported (off-diagonal entries must be 0, else REANN_E_UNSUPPORTED).
 *    pbc[3] != 0 marks a periodic axis.  Non-periodic axes must not be split.
 *  - Every array argument is caller-owned.  Inputs are copied before the call returns;
 *    outputs are written only when the call returns REANN_OK.  Handles are library-owned;
 *    every _free / _destroy accepts NULL.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory
 *    of the context's GPU.
 *  - No C++ exception crosses this boundary.  On failure the call returns a negative
 *    status and reann_last_error() describes it.
 *  - A context, nlist or plan must not be used by two threads at once.  reann_submit and
 *    reann_poll are thread-safe.
 *  - Plans and neighbour lists keep their context alive: reann_ctx_free releases the context
 *    once the last plan or list created on it has been freed.
 */
#ifndef REANN_H
#define REANN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t reann_status;
#define REANN_OK 0
#define REANN_PENDING 1
#define REANN_E_INVALID (-1)        /* NULL, n <= 0, T out of range, r_c mismatch, bad species, NaN, ... */
#define REANN_E_UNSUPPORTED (-2)    /* non-orthorhombic cell, (L, K) without a compiled kernel, ...     */
#define REANN_E_NOMEM (-3)          /* host or device allocation failed                                */
#define REANN_E_CAPACITY (-4)       /* request larger than a server's HBM budget                       */
#define REANN_E_DEVICE (-5)         /* HIP runtime error                                               */
#define REANN_E_UNKNOWN_TICKET (-6)
#define REANN_E_STATE (-7)          /* call out of order (e.g. backward before forward)               */

/* Arithmetic of the evaluation.  FP64: every step in double.  FP32: edge passes,
   densities and atomic NNs in float, positions and displacements formed in double,
   energy and virial sums in double.  BF16: as FP32 but the atomic-NN matrix products take
   bfloat16 operands with float accumulation.  FP8: the atomic-NN forward products take OCP
   e4m3 operands with float accumulation, one scale per weight matrix and per activation
   tensor, the activation scales calibrated once from an FP32 evaluation on the plan's first
   call (twice the largest magnitude seen maps to 448; larger values saturate); the adjoint
   products take bfloat16 operands. */
#define REANN_FP64 0
#define REANN_FP32 1
#define REANN_BF16 2
#define REANN_FP8 3

typedef struct reann_model reann_model;
typedef struct reann_ctx reann_ctx;
typedef struct reann_nlist reann_nlist;
typedef struct reann_plan reann_plan;
typedef struct reann_server reann_server;

/* Thread-local description of the last error on this thread; valid until the next call. */
const char *reann_last_error(void);

/* ------------------------------------------------------------------ model --
 * Model parameters (Sec. 2.1).  All arrays are host FP64 and copied.
 *   centres[K], alphas[K]   primitive Gaussians R_m(r) = exp(-alphas[m] (r - centres[m])^2)
 *   c0[n_species][K]        layer-0 orbital coefficients per element (dc^0/dr = 0)
 *   angular part            A(d) = (s dx)^lx (s dy)^ly (s dz)^lz, s = ang_scale, l <= L
 *   cutoff                  f_c(r) = (cos(pi r/r_c)/2 + 1/2)^2 for r < r_c, 0 beyond
 *   features                rho[l,(a,b)], a <= b, F = (L+1) K (K+1)/2, order l, a, b
 *   atomic NN dims          [F, hidden x n_hidden, out]: hidden layers z = W h + b, h = SiLU(z);
 *                           linear output.  Each NN is stored as W_1 [d1][d0] (row-major),
 *                           b_1 [d1], W_2, b_2, ...
 *   msg                     (T_max - 1) * n_species message NNs (out = K), ordered t-major
 *   en                      n_species energy NNs (out = 1); E_i = energy_scale * NN(rho_i^{T-1})
 *   form                    REANN_FORM_REANN: the above (Eqs. (1)-(2)).  REANN_FORM_RADIAL: a
 *                           second message form on the same per-layer exchange (Sec. 2.2, the
 *                           paragraph on other MPNNs that aggregate messages over neighbours):
 *                           L = 0, the K orbital sums themselves are the features,
 *                           x_i[m] = sum_j c_j[m] R_m(r_ij) f_c(r_ij) (F = K), and messages are
 *                           updated with a residual, c_i^{t+1} = c_i^t + NN^t(x_i^t);
 *                           E_i = energy_scale * NN(x_i^{T-1}).  FP64, FP32 and BF16 only.
 *                           REANN_FORM_DIAG: the literal reading of Eq. (1), only the squares,
 *                           rho[l,a] = sum_{|lambda|=l} l!/lambda! S[lambda,a]^2 (F = (L+1) K),
 *                           otherwise as REANN_FORM_REANN; runs on the per-layer NN kernels;
 *                           FP64, FP32 and BF16 only.
 * Supported (L, K): (2, 8), (2, 12), (1, 4), (2, 4) with REANN_FORM_REANN and REANN_FORM_DIAG;
 * (0, 8), (0, 12) with REANN_FORM_RADIAL; n_hidden 1..4; hidden <= 256. */
#define REANN_FORM_REANN 0
#define REANN_FORM_RADIAL 1
#define REANN_FORM_DIAG 2
typedef struct {
    int32_t n_species, L, K, T_max, n_hidden, hidden;
    double r_c, ang_scale, energy_scale;
    const double *centres, *alphas, *c0, *msg, *en;
    int32_t form;
} reann_model_desc;

reann_status reann_model_create(const reann_model_desc *desc, reann_model **out);
/* The same model from files.  spec_json_path: a JSON object with the members
 *   "format": "reann-model", "version": 1, n_species, L, K, T_max, n_hidden, hidden, r_c,
 *   ang_scale, energy_scale (numbers), optionally "form": "reann" (the default), "radial" or "diag",
 *   and "weights": path of the weight file (relative paths are taken from the spec's
 *   directory); other members (e.g. element names) are ignored.
 * The weight file is raw little-endian FP64: centres[K], alphas[K], c0[n_species][K], msg,
 * en, laid out as in reann_model_desc; its size must match the dimensions exactly.
 * REANN_E_INVALID for an unreadable or malformed spec or weight file. */
reann_status reann_model_load(const char *spec_json_path, reann_model **out);
/* Frees the model.  Plans (reann_plan_create) and servers made from it must be freed
 * first.  A context's cached state for reann_energy_forces may outlive the model: it is
 * never used again, since every model gets an id no later model reuses, even one created
 * at the same address. */
void reann_model_free(reann_model *m);

/* ---------------------------------------------------------------- context --
 * A context binds the library to one GPU and one HIP stream.  hip_stream may be NULL
 * (the library then creates a stream of default priority).  Device memory the
 * context needs is allocated on first use and kept until reann_ctx_free. */
reann_status reann_ctx_create(int32_t device, void *hip_stream, reann_ctx **out);
void reann_ctx_free(reann_ctx *ctx);

/* Options of an evaluation.  Zero-initialised = FP32, whole system, no skin, message
 * exchange.
 * exchange: what the subdomains exchange between MP layers.  REANN_EXCHANGE_MESSAGES (the
 *   paper's scheme, Sec. 2.2): ghosts receive their owners' messages c^{t+1} and send back the
 *   message adjoints.  REANN_EXCHANGE_NODE_FEATURES (the alternative the end of Sec. 2.2
 *   contrasts with it, node-feature communication): ghosts receive their owners' orbital
 *   sums S^t (NL K values instead of K), every subdomain evaluates the message NN for its
 *   ghosts as well as its locals, and the adjoints sent back are dE/dS^t.  Same results, more
 *   work and wider exchanges; FP64, FP32 and BF16 only. */
#define REANN_EXCHANGE_MESSAGES 0
#define REANN_EXCHANGE_NODE_FEATURES 1
typedef struct {
    int32_t precision;   /* REANN_FP64 / FP32 / BF16 / FP8                                 */
    int32_t decomp[3];   /* subdomains per axis; {0,0,0} or {1,1,1} = whole system          */
    double skin;         /* neighbour-list skin (A); the list is rebuilt when an atom has
                            moved more than skin/2 since the last build                    */
    int32_t exchange;    /* REANN_EXCHANGE_MESSAGES or REANN_EXCHANGE_NODE_FEATURES          */
} reann_opts;

/* ------------------------------------------------------------- neighbours --
 * reann_build_neighbors: neighbour list of every atom for cutoff r_c + skin (Sec. 2.2:
 * one list, reused by every MP layer), built on the GPU through the subdomain split
 * `decomp` (NULL = whole system).  The pair set is every copy (j, shift) of atom j
 * displaced by integer lattice vectors, (j, shift) != (i, 0), with
 *   d = (w_j + shift*L) - w_i,  fma(dz,dz, fma(dy,dy, dx*dx)) < (r_c+skin)^2   (FP64),
 * where w is the position wrapped into [0, L) on periodic axes by
 *   w = x - floor(x/L)*L, then +L if negative, then -L if >= L.
 * pos: host [n][3].  The result stays on the device; export it with reann_nlist_export.
 * Every list build (here and inside evaluations and plans) returns REANN_E_INVALID for
 * non-finite positions, |x| >= 1e9, or two copies closer than 1e-6 A (the direction of such
 * a pair, and so its force, is undefined). */
reann_status reann_build_neighbors(reann_ctx *ctx, const double *pos, int64_t n, const double cell[9],
                                   const int32_t pbc[3], double r_c, double skin, const int32_t decomp[3],
                                   reann_nlist **out);

/* Two-call export of the list in canonical order: each atom's row sorted by (j, shift).
   First call with row == NULL to get *n_pairs; then pass row[n+1], j[n_pairs],
   shift[n_pairs][3] (all host). */
reann_status reann_nlist_export(const reann_nlist *nl, int64_t *n_pairs, int64_t *row, int64_t *j,
                                int32_t *shift);

/* Sizes of a built list (each output may be NULL): atoms, ghost/image copies, stored pairs
   (rows of locals plus the rows of ghosts that the backward reads), pairs in the rows of
   the locals (the list proper). */
reann_status reann_nlist_info(const reann_nlist *nl, int64_t *n_atoms, int64_t *n_ghosts, int64_t *n_pairs,
                              int64_t *n_local_pairs);
void reann_nlist_free(reann_nlist *nl);

/* ----------------------------------------------------------- evaluation --
 * reann_energy_forces: one energy + force + virial evaluation (host pointers).
 *   pos[n][3], species[n] (0 <= s < n_species), r_c must equal the model's r_c,
 *   1 <= T <= model T_max.  opt may be NULL (FP32, whole system, skin 0).
 *   energy: host scalar (eV); forces: host [n][3] (eV/A) or NULL; virial: host [9] or NULL,
 *   W_ab = sum over directed edges of d_a f_b with f = -dE/dd (eV).
 * The context caches the plan of the last system: calling again with the same n, species,
 * cell, pbc, T and opts reuses it, and reuses the neighbour list while no atom has moved
 * more than skin/2. */
reann_status reann_energy_forces(reann_ctx *ctx, const reann_model *m, const double *pos, const int32_t *species,
                                 int64_t n, const double cell[9], const int32_t pbc[3], double r_c, int32_t T,
                                 const reann_opts *opt, double *energy, double *forces, double *virial);

/* reann_energy_forces_noalloc: reann_energy_forces for callers that cannot allocate device
 * memory (code that must not call hipMalloc, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and host-pointer conventions, but no device allocation
 * and no caching between calls: every device buffer of the evaluation (positions, neighbour
 * list, layer state, adjoint records, outputs) is carved from a static device array of 64 MiB
 * per GPU that the library holds from its load until the process ends.  That bounds the system
 * size: roughly 3,500 atoms at the Cu workload's shapes (r_c 6 A + 1 A skin, K = 12, T = 3) and
 * ~10,000 water atoms at r_c = 5 A, K = 8; larger inputs return REANN_E_CAPACITY.  Each call
 * builds the neighbour list afresh.  The model's device copies must already exist for this GPU
 * and precision (created by an earlier reann_energy_forces or reann_plan_create with the same
 * model), else REANN_E_STATE.  All calls on one GPU share its array: the library serialises
 * them within the process, and the array keeps the last call's contents (every buffer is
 * rewritten or cleared before use).  Calls on one GPU from several processes, or overlapping
 * work that another library places in the same array, race. */
reann_status reann_energy_forces_noalloc(reann_ctx *ctx, const reann_model *m, const double *pos,
                                         const int32_t *species, int64_t n, const double cell[9],
                                         const int32_t pbc[3], double r_c, int32_t T, const reann_opts *opt,
                                         double *energy, double *forces, double *virial);

/* Device-pointer path (used by the PyTorch autograd binding).  A plan fixes the system
 * (n, species, cell, pbc), the model, T and the options.  species is host [n].
 *   reann_plan_forward:  d_pos device FP64 [n][3]; writes d_energy (device FP64 scalar) and,
 *                        if not NULL, d_atom_energy (device FP64 [n]).  Enqueued on hip_stream
 *                        (NULL = HIP's null stream, which is also PyTorch's default stream);
 *                        checks the skin rule on that stream and rebuilds the neighbour list
 *                        when an atom has moved more than skin/2 (unless the plan's list
 *                        policy leaves that to the caller, below).  On a built list the
 *                        forward is queued behind the check and the call waits for the check
 *                        alone (the forward runs meanwhile); after a rebuild the forward is
 *                        queued again, so the outputs are those of the rebuilt list.
 *   reann_plan_backward: gradient of E w.r.t. positions after a forward: d_grad_energy is a
 *                        device FP64 scalar g (NULL = 1); writes d_forces = -g dE/dx (device FP64
 *                        [n][3]) and, if not NULL, d_virial = g W (device FP64 [9]).  Enqueued
 *                        on hip_stream (NULL = null stream).  REANN_E_STATE if no forward
 *                        preceded it. */
reann_status reann_plan_create(reann_ctx *ctx, const reann_model *m, const int32_t *species, int64_t n,
                               const double cell[9], const int32_t pbc[3], int32_t T, const reann_opts *opt,
                               reann_plan **out);
reann_status reann_plan_forward(reann_plan *p, const double *d_pos, double *d_energy, double *d_atom_energy,
                                void *hip_stream);
reann_status reann_plan_backward(reann_plan *p, const double *d_grad_energy, double *d_forces, double *d_virial,
                                 void *hip_stream);
void reann_plan_free(reann_plan *p);

/* Neighbour-list upkeep of a plan (Sec. 2.2: one list for r_c + skin, reused while every atom
 * stays within skin/2 of where it was built).
 *   reann_plan_set_list_policy: auto_check = 1 (the default): every reann_plan_forward checks
 *     the skin rule (one wait for the check) and rebuilds the list when needed.
 *     auto_check = 0: forwards use the current list as it is and make no host synchronisation
 *     and no device allocation, so a forward + backward can be captured in a HIP graph and
 *     replayed; the caller keeps the list valid with reann_plan_update_list (for instance every
 *     few MD steps, or when its own bound on the displacement since the last build reaches
 *     skin/2).  A forward before any list has been built returns REANN_E_STATE.
 *   reann_plan_update_list: the skin check at positions d_pos (device FP64 [n][3]) on
 *     hip_stream, and a rebuild when it fails or no list exists; synchronises that stream.
 *     rebuilt (host int32, may be NULL) is set to 1 after a rebuild, else 0.  A rebuild may
 *     move the plan's device buffers, so a graph captured before it must be captured again. */
reann_status reann_plan_set_list_policy(reann_plan *p, int32_t auto_check);
reann_status reann_plan_update_list(reann_plan *p, const double *d_pos, void *hip_stream, int32_t *rebuilt);

/* Weights of the atomic energies in the plan's energy: E = sum_i w_i E_i, and the backward
 * gives the gradient of that weighted sum (forces, virial).  w: host [n] in caller order,
 * copied; NULL restores w_i = 1.  Atomic energies (d_atom_energy) stay unweighted.  Used to
 * evaluate a subdomain together with copies of atoms it does not own, counting only its own
 * atoms' energies (the extended-halo scheme, where each subdomain recomputes its halo). */
reann_status reann_plan_set_energy_weights(reann_plan *p, const double *w);

/* Number of forwards run on the plan so far (0 before the first).  A backward always uses the
 * state of the plan's most recent forward; a caller that keeps several forwards alive (e.g. an
 * autograd graph) records the number after each forward and compares it before the backward
 * to detect that another forward has replaced that state.  gen: host scalar. */
reann_status reann_plan_generation(const reann_plan *p, uint64_t *gen);

/* Intermediate values of the last forward, for layer-by-layer checks, copied to host in
 * the caller's atom order:  what = 0: orbital sums S^t [n][NL][K] (NL = (L+1)(L+2)(L+3)/6,
 * components ordered by l, then lx descending, then ly descending); 1: messages c^t [n][K];
 * 2: atomic energies [n] (t ignored).  Synchronises the stream. */
reann_status reann_plan_get(reann_plan *p, int32_t what, int32_t t, double *host_out);
/* The two device-pointer steps under their short names: reann_forward_dev is
 * reann_plan_forward without per-atom energies, reann_backward_dev is reann_plan_backward. */
reann_status reann_forward_dev(reann_plan *p, const double *d_pos, double *d_energy, void *hip_stream);
reann_status reann_backward_dev(reann_plan *p, const double *d_grad_energy, double *d_forces, double *d_virial,
                                void *hip_stream);

/* Kernel time per phase, measured with HIP events recorded on the evaluation stream at
 * phase boundaries while timing is enabled (reann_plan_set_timing), accumulated over every
 * forward+backward since the previous reann_plan_timing call.  REANN_N_PHASES phases:
 *   [0] neighbour-list reuse check and rebuilds, [1] edge forward (orbital sums),
 *   [2] density contraction, [3] atomic NN forward, [4] ghost exchange,
 *   [5] atomic NN adjoint, [6] density adjoint, [7] edge adjoint, centre role,
 *   [8] edge adjoint, neighbour role, [9] other (refresh, compaction, seeds, reductions,
 *   output).
 * ms: host [REANN_N_PHASES] milliseconds; launches (host [REANN_N_PHASES] or NULL): kernel
 * launches of the phases that time one kernel type ([1], [2], [6], [7], [8], and [3], [5]
 * when the atomic NNs run fused; 0 elsewhere; [0] counts rebuilds); steps (or NULL):
 * backward passes covered.  Synchronises on the last event and resets the accumulators. */
#define REANN_N_PHASES 10
reann_status reann_plan_set_timing(reann_plan *p, int32_t enable);
reann_status reann_plan_timing(reann_plan *p, double *ms, int64_t *launches, int64_t *steps);

/* ---------------------------------------------------------------- serving --
 * Continuous-batching server: many independent systems stay resident on the device
 * (positions, velocities, neighbour lists, features); requests that arrive while others
 * run are admitted as batch slots and HBM budget free up.  Up to 8 requests are in flight at
 * once, each on its own stream, so steps of different systems overlap on the device; one
 * request per system is in flight at a time (a velocity-Verlet step needs the previous
 * forces).  When the budget is exhausted, idle resident systems are evicted (least recently
 * used first, their state copied back to the host), else the request waits.  A step replays
 * a captured HIP graph while the neighbour list is unchanged.  Results do not depend on which
 * other requests are in flight.
 *   hbm_budget_bytes  device memory the resident systems may use (0 = 3/4 of free memory);
 *                     reann_system_add returns REANN_E_CAPACITY for a system that can never fit.
 *   max_batch_atoms   cap on the total atoms of the requests in flight at once (0 = 262144);
 *                     a request that would exceed it waits (a lone request always runs).
 *                     Requests are not packed into shared launches: each runs its own
 *                     system's kernels on its own stream, up to 8 at a time.
 *   precision, T, skin as in reann_opts.  use_graph != 0 replays, once the step's positions are
 *   in place and its list checked, one captured HIP graph per system (forward, backward, the
 *   rest of a velocity-Verlet step, the result copy), captured again when the list is rebuilt
 *   or the request kind, time step or skipped outputs change.
 *   thermostat_K, thermostat_tau_fs: both > 0 ends every REANN_REQ_VV_STEP with a Berendsen
 *   velocity rescaling (Berendsen et al., J. Chem. Phys. 81, 3684 (1984)) toward
 *   thermostat_K with time constant thermostat_tau_fs: v *= sqrt(1 + (dt / tau)(T0 / T - 1)),
 *   T = 2 K / (3 n k_B) from the kinetic energy K after the step; 0 (either) = constant energy. */
typedef struct {
    int64_t hbm_budget_bytes;
    int64_t max_batch_atoms;
    int32_t precision;
    int32_t T;
    double skin;
    int32_t use_graph;
    int32_t device;
    double thermostat_K;
    double thermostat_tau_fs;
    int32_t decomp[3];       /* subdomains per axis for every system ({0,0,0} or {1,1,1} = whole
                                system), as in reann_opts: each system is evaluated split, with the
                                per-layer ghost exchange, and every skin-rule rebuild reassigns its
                                atoms to subdomains by their current positions (atom migration) */
    int32_t thermostat;      /* REANN_THERMO_BERENDSEN or REANN_THERMO_CSVR (used when
                                thermostat_K > 0 and thermostat_tau_fs > 0)                     */
    uint64_t seed;           /* CSVR: seed of each system's random stream (mixed with its id)   */
} reann_server_opts;

/* Thermostats of REANN_REQ_VV_STEP (applied at the end of the step, from the kinetic energy K
 * after it, N_f = 3 n, K_0 = N_f k_B thermostat_K / 2, c = exp(-dt / thermostat_tau_fs)):
 *  BERENDSEN  v *= sqrt(1 + (dt / tau)(K_0 / K - 1))   (Berendsen et al., J. Chem. Phys. 81, 3684
 *             (1984)); relaxes K to K_0 but suppresses its fluctuations, so it does not sample the
 *             canonical ensemble.
 *  CSVR       stochastic velocity rescaling (Bussi, Donadio and Parrinello, J. Chem. Phys. 126,
 *             014101 (2007)): v *= sqrt(K' / K) with
 *             K' = K + (1 - c)(K_0 (R^2 + S) / N_f - K) + 2 R sqrt(c (1 - c) K K_0 / N_f),
 *             R ~ N(0, 1) and S ~ chi^2 with N_f - 1 degrees of freedom drawn on the host from the
 *             system's seeded stream; samples the canonical (NVT) ensemble. */
#define REANN_THERMO_BERENDSEN 0
#define REANN_THERMO_CSVR 1

#define REANN_REQ_EVAL 0      /* evaluate E, F, W at the given positions (pos required)        */
#define REANN_REQ_VV_STEP 1   /* one velocity-Verlet step of dt_fs (pos ignored), then E, F, W  */

/* Result vectors a request may leave on the device (reann_request.skip_outputs, or-ed). */
#define REANN_OUT_FORCES 1
#define REANN_OUT_POSITIONS 2
#define REANN_OUT_VELOCITIES 4

typedef struct {
    uint64_t sys_id;
    int32_t kind;
    double dt_fs;
    const double *pos;        /* host [n][3] for REANN_REQ_EVAL, copied by reann_submit */
    int32_t skip_outputs;     /* REANN_OUT_* vectors not copied back to the host (0 = all three
                                 come back); energy, virial and kinetic energy always do.  A
                                 dynamics run that reads vectors only now and then skips them on
                                 the other steps.  Other bits: REANN_E_INVALID.              */
} reann_request;

typedef struct {
    double energy;
    double virial[9];
    double *forces;           /* caller-owned host [n][3], or NULL to skip                   */
    double *positions;        /* caller-owned host [n][3], or NULL: positions after the step */
    int64_t t_submit_ns, t_done_ns;   /* CLOCK_MONOTONIC                                    */
    reann_status status;      /* status of the request itself                              */
    double kinetic;           /* REANN_REQ_VV_STEP: kinetic energy (eV) of the velocities after
                                 the step (after any rescaling); 0 for REANN_REQ_EVAL        */
    double *velocities;       /* caller-owned host [n][3] (A/fs), or NULL: the system's velocities
                                 after the request (after any rescaling)                     */
} reann_result;

reann_status reann_server_create(const reann_model *m, const reann_server_opts *opt, reann_server **out);
/* masses: host [n_species] in amu, used by REANN_REQ_VV_STEP (NULL = no dynamics). */
reann_status reann_server_set_masses(reann_server *s, const double *masses_amu);
reann_status reann_system_add(reann_server *s, const int32_t *species, int64_t n, const double cell[9],
                              const int32_t pbc[3], const double *pos, const double *vel, uint64_t *sys_id);
reann_status reann_submit(reann_server *s, const reann_request *req, uint64_t *ticket);
/* Non-blocking: REANN_PENDING while running, REANN_OK when res is filled (the ticket is then
   released), or a negative status.  A non-NULL res->forces, positions or velocities for a vector
   the request skipped returns REANN_E_INVALID and keeps the result for another poll.  A request that fails for its inputs (e.g. REANN_E_INVALID
   from the neighbour build when the step brought two atoms within 1e-6 A) fails alone: its
   system's device state is dropped, later requests for that system return REANN_E_STATE, and
   the server keeps serving the others.  A device error fails every request and the server.
   Test hook: with the environment variable REANN_SERVER_FAULT_TICKET=k set when the server is
   created, request ticket k is refused as if its inputs were invalid. */
reann_status reann_poll(reann_server *s, uint64_t ticket, reann_result *res);
/* Statistics, host [REANN_N_SERVER_STATS]: [0] engine rounds that admitted at least one
   request, [1] requests completed, [2] atoms evaluated, [3] HIP-graph replays, [4] admissions
   deferred for the HBM budget, [5] device bytes held by resident systems, [6] neighbour-list
   builds (first builds and skin-rule rebuilds), [7] host nanoseconds the launcher threads spent
   enqueuing steps (launches, list checks and rebuilds, copies; summed over the threads), [8] of
   which in HIP-graph launches,
   [9] host nanoseconds spent unpacking finished requests, [10] of [7] in neighbour-list
   builds, [11] of [7] in capturing and instantiating HIP graphs, [12] skin checks on the
   device (steps whose list the previous step's prediction or the displacement bound did not
   decide), [13] of [7] in them, [14] velocity-Verlet steps whose list the previous step's
   prediction decided (it computes the displacement that the next drift of the same dt gives). */
#define REANN_N_SERVER_STATS 15
reann_status reann_server_stats(reann_server *s, int64_t *stats);
void reann_server_destroy(reann_server *s);

#ifdef __cplusplus
}
#endif
#endif /* REANN_H */
