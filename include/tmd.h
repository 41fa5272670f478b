/*
 * tmd.h -- C ABI of libtmd.so: TensorMD energy, force and virial evaluation
 * on one AMD Instinct MI355X (gfx950).
 *
 * The computation follows the TensorMD paper (arXiv 2310.08439):
 *   neighbour table of typed neighbours (Sec. III.A, the R_abc / D_abcx tensors)
 *   -> radial functions H_abck times moment tensors M_abcd of the neighbour unit
 *      vectors, contracted to G_abkm = sigma(T_dm (H_abck M_abcd)^2)
 *      (Sec. III.A, eqns T_dm, tensor_formalism, sigma_function)
 *   -> per-element MLP atomic energies E_a, E = sum_a E_a (Sec. III.A)
 *   -> forces by the adjoint chain P', U, V, F1, F2 and ScatterSum
 *      (Sec. III.A, eqns dP_abkd, U_abck, F1_abcx, F2_abcx), plus the virial.
 *
 * Conventions
 *   Units: Angstrom, eV, amu, fs.
 *   Boxes are orthorhombic and periodic in x, y and z.
 *   Pair vector D = x_j + n*L - x_i (neighbour minus centre, n the periodic image).
 *   Radial functions h_k(R) = exp(-eta_k (R - mu_k)^2) * f_c(R) with the cosine
 *   cutoff f_c(R) = (cos(pi R / rcut) + 1)/2 for R < rcut and 0 beyond.
 *   Descriptor feature index ((b*K + k)*(M+1) + m), b = species of the neighbour.
 *   Virial W_ab = -sum over pairs of D_a dE/dD_b, reported as (xx, yy, zz, xy, xz, yz).
 *
 * Ownership
 *   The caller owns every pointer argument; pointers marked "device" are HIP
 *   device allocations (for instance torch tensors), pointers marked "host" are
 *   host memory.  The library owns only the opaque handles and frees them in
 *   the matching *_destroy.  No call keeps a caller pointer after it returns.
 *   All device work is enqueued on the context's stream.  Calls that write a
 *   host output synchronise that stream before returning.
 *
 * Errors
 *   Every call returns a tmd_status; nothing throws across the ABI.
 *   tmd_last_error(ctx) returns a message for the last failure on ctx.
 *
 * Threads
 *   A context is used by one host thread at a time.
 */
#ifndef TMD_H
#define TMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TMD_OK = 0,
    TMD_ERR_INVALID_ARGUMENT = 1,  /* null pointer, bad size, species out of range, bad model shape */
    TMD_ERR_CAPACITY = 2,          /* a neighbour list row would exceed the list capacity */
    TMD_ERR_OUT_OF_MEMORY = 3,     /* device allocation failed */
    TMD_ERR_DEVICE = 4,            /* a HIP runtime call failed */
    TMD_ERR_NUMERICAL = 5,         /* non-finite position or two atoms at distance 0 */
    TMD_ERR_NOT_READY = 6,         /* asynchronous result not available yet */
    TMD_ERR_REJECTED = 7           /* request can never be admitted (larger than the budget) */
} tmd_status;

/* Arithmetic of the MLP stage.  Descriptors and the adjoint always run in
 * FP32 and totals in FP64 (compensated). */
typedef enum {
    TMD_FP32 = 0,      /* MLP GEMMs on FP32 MFMA, FP32 accumulation */
    TMD_BF16_MLP = 1   /* MLP GEMM operands rounded to BF16 (nearest-even), FP32 accumulation */
} tmd_precision;

typedef enum { TMD_ACT_TANH = 0, TMD_ACT_SQUAREPLUS = 1 } tmd_activation;

typedef struct tmd_context tmd_context;
typedef struct tmd_model tmd_model;
typedef struct tmd_nlist tmd_nlist;

/* One periodic system.  pos: device, [n_atoms][3] FP64; species: device,
 * [n_atoms] int32 in [0, n_species). */
typedef struct {
    int64_t n_atoms;
    const double* pos;
    const int32_t* species;
    double box[3];
} tmd_system_view;

#define TMD_MAX_HIDDEN 4

/* Shape of a model (Sec. III.A and the tensor ranges of Table I).
 *   n_species   S, 1..8 (the neighbour-species index b and the MLP selector)
 *   n_radial    K, 1..128
 *   max_moment  M, 0..3 (D = 1, 4, 10, 20 moment components)
 *   n_hidden    1..4 hidden layers of widths hidden[0..n_hidden-1], each 1..128
 *   activation  tmd_activation of the hidden layers; the output layer is linear
 *   rcut        cutoff radius (A), > 0
 *   mu, eta     host, [K] FP64: Gaussian centres (finite) and widths (finite, >= 0) of h_k.
 * Internally the kernels run K rounded up to 4, 6 or 8 times a power of two
 * and every hidden layer at the widest width rounded up to 32, 64 or 128; the
 * extra radial functions and hidden units meet zero weights and change no
 * result, but cost their share of the work (K = 10 runs 12 radial functions). */
typedef struct {
    int32_t n_species;
    int32_t n_radial;
    int32_t max_moment;
    int32_t n_hidden;
    int32_t hidden[TMD_MAX_HIDDEN];
    int32_t activation;
    int32_t reserved;
    double rcut;
    const double* mu;
    const double* eta;
} tmd_model_spec;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL for the legacy default stream). */
tmd_status tmd_context_create(int device, void* hip_stream, tmd_context** out);
void tmd_context_destroy(tmd_context* ctx);
/* Re-target the context at another stream of the same device. */
tmd_status tmd_context_set_stream(tmd_context* ctx, void* hip_stream);
/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char* tmd_last_error(const tmd_context* ctx);

/* Per-kernel timing.  While enabled, every kernel the context launches is
 * bracketed by two HIP events on the context's stream.  tmd_profile_read
 * synchronises, writes up to max_kernels entries (name[i] is a 32-byte
 * NUL-terminated field of the host array names, total_ms[i] the summed
 * duration, count[i] the number of launches) and returns the number of
 * distinct kernels.  tmd_profile_reset clears the totals. */
tmd_status tmd_profile_enable(tmd_context* ctx, int on);
tmd_status tmd_profile_reset(tmd_context* ctx);
int32_t tmd_profile_read(tmd_context* ctx, int32_t max_kernels, char* names, double* total_ms, int64_t* count);

/* ---------------------------------------------------------------- model */

/* Upload a model.  params: host FP32, per species in species order, each block
 * laid out layer by layer as W_l row-major [out][in] followed by b_l [out],
 * ending with the output layer w [1][hidden] and its bias [1].  Block length:
 * sum_l (w_l * w_{l-1} + w_l) + hidden + 1 with w_0 = S*K*(M+1). */
tmd_status tmd_model_create(tmd_context* ctx, const tmd_model_spec* spec, const float* params, tmd_model** out);
/* Replace the weights of an existing model (same layout as tmd_model_create). */
tmd_status tmd_model_set_params(tmd_model* model, const float* params);
tmd_status tmd_model_set_precision(tmd_model* model, tmd_precision precision);
/* Copy the current weights (host FP32, same layout as tmd_model_create) into
 * params; reflects every tmd_train_step applied so far.  Synchronises. */
tmd_status tmd_model_get_params(const tmd_model* model, float* params);
/* Tabulated radial functions (Sec. III.B: the radial tensor H and its
 * derivative H' interpolated from a 1-D table, with the cutoff folded into the
 * table and nothing evaluated past rcut).  The paper's rational-interpolation
 * formula is not printed; this uses piecewise cubic Hermite interpolation:
 * nodes r_j = j * delta with delta = rcut / ceil(rcut / dr) (so rcut is a
 * node), node values and derivatives of h_k = exp(-eta_k (R - mu_k)^2) f_c(R)
 * computed exactly in FP64, both forced to 0 at r = 0 as the paper does, and
 * stored per interval as four FP32 polynomial coefficients, interval-major
 * ([interval][k], 16 bytes per entry).  h_k' is the derivative of the same
 * cubic, so forces stay the exact gradient of the tabulated energy.
 * dr = 0 returns to direct evaluation.  The table serves tmd_descriptors,
 * tmd_energy_forces(_async), tmd_md_* and tmd_serve_*; tmd_train_step rejects a
 * tabulated model (training uses the exact functions).
 * Errors: dr < 0, not finite, > rcut, or more than 2^20 intervals ->
 * TMD_ERR_INVALID_ARGUMENT (the model keeps its previous mode); allocation ->
 * TMD_ERR_OUT_OF_MEMORY.  Synchronises the model's stream; must not run while
 * other work that uses the model is in flight. */
tmd_status tmd_model_tabulate(tmd_model* model, double dr);
/* Node spacing delta of the table in use (0 for direct evaluation). */
double tmd_model_tab_spacing(const tmd_model* model);
/* Number of floats per species block of params. */
int64_t tmd_model_params_per_species(const tmd_model* model);
int32_t tmd_model_n_features(const tmd_model* model);
void tmd_model_destroy(tmd_model* model);

/* ---------------------------------------------------------------- neighbour list */

/* A neighbour list for up to n_atoms atoms with room for at least `capacity`
 * neighbours of each species per atom (rounded up to a multiple of 4;
 * tmd_nlist_capacity reports the value used). */
tmd_status tmd_nlist_create(tmd_context* ctx, int64_t n_atoms, int32_t n_species, int32_t capacity,
                            tmd_nlist** out);
void tmd_nlist_destroy(tmd_nlist* nl);

/* Cell-list neighbour search under periodic boundaries (the binning search of
 * Sec. IV.D).  Lists every (j, n) != (i, 0) with |x_j + n*L - x_i| < rcut + skin,
 * evaluated in FP64 on positions wrapped into [0, L); periodic self-images are
 * included.  On TMD_ERR_CAPACITY *required_capacity (host, may be NULL) is the
 * smallest capacity that would fit; the list is then unusable.  Synchronises. */
tmd_status tmd_build_neighbors(tmd_context* ctx, const tmd_system_view* sys, double rcut, double skin,
                               tmd_nlist* nl, int32_t* required_capacity);

/* Copy the list out, in original atom numbering.  Device outputs:
 * nbr [n][S][capacity] int32 (-1 padding), img [n][S][capacity][3] int32
 * periodic image, cnt [n][S] int32 entries per neighbour species.
 * Order within a row is unspecified. */
tmd_status tmd_nlist_export(tmd_context* ctx, const tmd_nlist* nl, int32_t* nbr, int32_t* img, int32_t* cnt);
int32_t tmd_nlist_capacity(const tmd_nlist* nl);

/* Totals of the last build: *total_pairs (host) = number of list entries,
 * *max_row (host) = longest per-species row.  Synchronises. */
tmd_status tmd_nlist_stats(tmd_context* ctx, const tmd_nlist* nl, int64_t* total_pairs, int32_t* max_row);

/* ---------------------------------------------------------------- evaluation */

/* Descriptors G_abkm (Sec. III.A, eqns tensor_formalism and sigma_function:
 * P = sum_c H M, S = T P^2, G = sqrt(S) for m = 0 and S otherwise) for the
 * positions in sys, using a list built by tmd_build_neighbors for the same
 * atoms (positions may have moved by less than skin/2 since).
 * G: device, [n][S*K*(M+1)] FP32, original atom order, feature index
 * ((b*K + k)*(M+1) + m).  Errors as tmd_energy_forces.  Does not synchronise. */
tmd_status tmd_descriptors(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys,
                           const tmd_nlist* nl, float* G);

/* Energy, forces and virial (Sec. III.A).  energy: host FP64 total (Neumaier-
 * compensated sum of atomic energies); atom_energy: device [n] FP32 or NULL;
 * forces: device [n][3] FP32 (F = -dE/dx); virial6: host FP64 [6] or NULL.
 * With a list built with a skin, each call first copies the list's rows
 * keeping the entries within rcut at the current positions (scratch owned by
 * the list, as large as its rows, allocated at the first such call; an
 * allocation failure returns TMD_ERR_OUT_OF_MEMORY).  Synchronises the stream. */
tmd_status tmd_energy_forces(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys,
                             const tmd_nlist* nl, double* energy, float* atom_energy, float* forces,
                             double* virial6);

/* Same as tmd_energy_forces but leaves the totals on the device and does not
 * synchronise: totals7 is device FP64 [7] = (E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz). */
tmd_status tmd_energy_forces_async(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys,
                                   const tmd_nlist* nl, double* totals7, float* atom_energy, float* forces);

/* Energy, forces and virial of several systems in one launch chain (the
 * continuous batching of many small systems a server sees; same quantities as
 * tmd_energy_forces_async, Sec. III.A).  systems[s] and lists[s] as for
 * tmd_energy_forces_async (each list built for its system, positions moved by
 * less than skin/2 since; the lists are only read); 1..4096 systems.  The
 * lists are merged into one over the concatenated atoms (each system padded to
 * a multiple of 256 atoms; a pair's image shift uses its system's box) and the
 * descriptor, MLP and adjoint run once over all of them, with the adjoint's
 * force scatter by device atomics (fixed point, so each system's forces do
 * not depend on what it was batched with).  Outputs: totals7 device FP64
 * [n_systems][7] = (E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz) per system, summed in
 * FP64 with compensation; forces[s] device [n_s][3] FP32, system s's atom
 * order.  Errors: as tmd_energy_forces_async for each system; a null array or
 * a count outside 1..4096 -> TMD_ERR_INVALID_ARGUMENT.  Does not synchronise
 * (the host table of systems is copied before the call returns). */
tmd_status tmd_energy_forces_batch(tmd_context* ctx, const tmd_model* model, int32_t n_systems,
                                   const tmd_system_view* systems, const tmd_nlist* const* lists, double* totals7,
                                   float* const* forces);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as tmd_energy_forces_async, with every intermediate (descriptors,
 * their gradient, the P tensors, atomic energies, force accumulators, virial
 * and energy partials) in one scratch array that the library holds in device
 * memory, tmd_noalloc_scratch_bytes() = 64 MiB per device, for the life of the
 * process.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine) and does not synchronise; the caller still passes the
 * outputs: totals7 device FP64 [7] = (E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz),
 * atom_energy device [n] FP32 or NULL, forces device [n][3] FP32.
 * The list must be built with rlist = rcut (no skin; a skin list needs
 * pruned-row memory); per-kernel timing is suspended during the call.
 * Errors: as tmd_energy_forces_async; a system whose intermediates need more
 * than the scratch (about 2.7 KB per atom for 96 features, K = 12, two
 * species: roughly 24,000 atoms) -> TMD_ERR_INVALID_ARGUMENT with the size
 * it needs.  All calls on one device share its scratch and its contents
 * persist between calls: calls that overlap on one device (other streams,
 * other host threads, other contexts) race and must not be issued. */
tmd_status tmd_energy_forces_noalloc(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys,
                                     const tmd_nlist* nl, double* totals7, float* atom_energy, float* forces);
/* Size of the per-device scratch array of tmd_energy_forces_noalloc, in bytes. */
int64_t tmd_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- training (force matching) */

/* Force matching is not part of the paper's method (its potentials were
 * trained elsewhere); it trains the same per-element MLP on energy and force
 * labels.  Over a batch of B periodic systems with N atoms in total,
 *   L = (1/B) sum_s ((E_s - Ehat_s)/N_s)^2 + lambda/(3N) sum_i |F_i - Fhat_i|^2,
 * whose parameter gradient needs the derivative of the forces with respect to
 * the weights: the forces' residual r = dL/dF is pushed through the
 * descriptors as a tangent (forward mode, w_i = d/de G_i(x + e r)) and the
 * network is differentiated twice (forward-over-reverse), so that
 * dL/dtheta = sum_i [e_i dE_i/dtheta - d(grad_G E_i . w_i)/dtheta] with
 * e_i = (2/B)(E_s - Ehat_s)/N_s^2 for the atoms of system s. */
typedef struct tmd_batch tmd_batch;

typedef enum { TMD_OPT_ADAM = 0, TMD_OPT_SGD = 1 } tmd_optimizer;

/* lambda: force-term weight (0.1 in the reference setup); lr: step size, 0
 * computes loss and gradient without touching the weights; beta1, beta2, eps:
 * Adam constants (0.9, 0.999, 1e-8); optimizer: tmd_optimizer. */
typedef struct {
    double lambda;
    double lr;
    double beta1;
    double beta2;
    double eps;
    int32_t optimizer;
    int32_t reserved;
} tmd_train_opts;

/* Copy a labelled batch to the device and prepare it for training with
 * models of the descriptor shape of `model` (S, K, M, rcut, mu, eta).
 * System s holds atoms sys_off[s] .. sys_off[s+1]-1 (host int64 [B+1],
 * sys_off[0] = 0) in the box boxes[3s .. 3s+2] (host FP64 [B][3]).
 * pos: device FP64 [N][3]; species: device int32 [N]; energy_labels: host FP64
 * [B]; force_labels: device FP32 [N][3].  Builds each system's neighbour list
 * with the cell-list search (at least `capacity` entries per row, 0 for the
 * default; grown as needed), stores the pair vectors D, the descriptors G and
 * the tensors P (fixed for the batch, since training changes only the MLP).
 * Synchronises. */
tmd_status tmd_batch_create(tmd_context* ctx, const tmd_model* model, int32_t n_systems, const int64_t* sys_off,
                            const double* pos, const int32_t* species, const double* boxes,
                            const double* energy_labels, const float* force_labels, int32_t capacity,
                            tmd_batch** out);
void tmd_batch_destroy(tmd_batch* batch);

/* One training step on the whole batch: energies and forces of the current
 * model (FP32, the model's precision setting is ignored), the loss, its
 * gradient and, when opts->lr > 0, one Adam or SGD update of the weights in
 * place (Adam state lives in the model).  loss: host FP64 [3] = (L, energy
 * term, force term) before the update; grad: device FP32 [S * params per
 * species] in the tmd_model_create layout, or NULL.  Synchronises. */
tmd_status tmd_train_step(tmd_context* ctx, tmd_model* model, const tmd_batch* batch, const tmd_train_opts* opts,
                          double* loss, float* grad);

/* Intermediate results of the last tmd_train_step (or of tmd_batch_create for
 * TMD_BATCH_G), in the batch's atom order, copied to device `out`:
 *   TMD_BATCH_G        [N][F] descriptors
 *   TMD_BATCH_ENERGY   [N]    atomic energies
 *   TMD_BATCH_FORCES   [N][3] forces
 *   TMD_BATCH_RESIDUAL [N][3] r = dL/dF
 *   TMD_BATCH_TANGENT  [N][F] descriptor tangents w along r */
typedef enum {
    TMD_BATCH_G = 0,
    TMD_BATCH_ENERGY = 1,
    TMD_BATCH_FORCES = 2,
    TMD_BATCH_RESIDUAL = 3,
    TMD_BATCH_TANGENT = 4
} tmd_batch_field;
tmd_status tmd_batch_read(tmd_context* ctx, const tmd_batch* batch, int32_t field, float* out);

/* ---------------------------------------------------------------- molecular dynamics */

/* Molecular dynamics of one system (the MD protocol of Sec. IV.D: NVT at
 * 300 K, 1 fs steps, a 1 A skin rebuilt every 5 steps, thermodynamic output
 * every 10 steps).  Velocity Verlet with accelerations 9.648533e-3 F/m A/fs^2;
 * for NVT a Nose-Hoover thermostat (the paper does not name one): a single
 * variable xi of mass Q = 3N kB T tau^2 in the symmetric Trotter splitting
 *   half thermostat step: xi += dt/4 G; v *= exp(-xi dt/2); eta += xi dt/2; xi += dt/4 G
 *   velocity Verlet step
 *   half thermostat step,
 * G = (2 KE - 3N kB T)/Q.  Positions stay FP64 on the device and are never
 * wrapped (the list build wraps them). */
typedef struct tmd_md tmd_md;

typedef enum { TMD_ENSEMBLE_NVE = 0, TMD_ENSEMBLE_NVT_NOSE_HOOVER = 1 } tmd_ensemble;

/* dt_fs > 0; temperature_K and tau_fs > 0 for NVT; skin >= 0 (A);
 * rebuild_every > 0: rebuild the list every that many steps (the caller
 * guarantees that no atom moves more than skin/2 in between); 0: rebuild when
 * an atom has moved more than skin/2 since the last build (one host
 * synchronisation per step).  With a skin, the force evaluations walk rows
 * pruned to rcut + skin/5, rebuilt on the device whenever the displacement
 * since the build could have brought a dropped pair inside rcut. */
typedef struct {
    double dt_fs;
    double temperature_K;
    double tau_fs;
    double skin;
    int32_t ensemble;
    int32_t rebuild_every;
} tmd_md_opts;

/* One line of thermodynamic output.  Energies in eV, temperature
 * T = 2 KE / (3N kB), pressure tensor diagonal p_aa = (2 KE_aa + W_aa)/V in GPa
 * and P its mean; conserved = PE + KE (+ Q xi^2/2 + 3N kB T eta for NVT);
 * rebuilds = list builds so far (including the first). */
typedef struct {
    int64_t step;
    double time_fs;
    double epot;
    double ekin;
    double etotal;
    double temperature_K;
    double pressure_GPa;
    double pxx_GPa;
    double pyy_GPa;
    double pzz_GPa;
    double volume_A3;
    double conserved;
    double xi;
    int32_t rebuilds;
    int32_t reserved;
} tmd_thermo;

/* Start MD from the positions and species of sys (device, copied), host FP64
 * masses per species [S] (amu) and device FP64 velocities [n][3] (copied; NULL
 * for zero).  Builds the list and evaluates the initial forces.  model must
 * outlive the handle.  Synchronises. */
tmd_status tmd_md_create(tmd_context* ctx, const tmd_model* model, const tmd_system_view* sys, const double* masses,
                         const double* velocities, const tmd_md_opts* opts, tmd_md** out);
/* Advance n_steps.  When thermo_every > 0, a tmd_thermo record is written to
 * the host array thermo (room for thermo_capacity records) at every step index
 * divisible by thermo_every (step 0 on the first call included); *n_thermo
 * (nullable) receives the number written.  Synchronises. */
tmd_status tmd_md_run(tmd_md* md, int64_t n_steps, int32_t thermo_every, tmd_thermo* thermo, int32_t thermo_capacity,
                      int32_t* n_thermo);
/* Copy the current positions / velocities to device arrays [n][3] (nullable). */
tmd_status tmd_md_read(tmd_md* md, double* pos, double* vel);
/* Host FP64 [2] = (xi, eta) of the thermostat. */
tmd_status tmd_md_thermostat_state(tmd_md* md, double* xi_eta);
void tmd_md_destroy(tmd_md* md);

/* ---------------------------------------------------------------- serving */

/* A persistent request loop over resident systems (the MD protocol of
 * Sec. IV.D, one velocity-Verlet NVE step being a full energy-and-force
 * evaluation).  Systems are registered once and stay on the device: positions
 * and velocities (FP64), species and, while memory allows, their neighbour
 * list.  Requests are served by max_slots worker threads, each with its own
 * HIP stream and workspace, so requests admitted together run concurrently on
 * the device; a request is admitted when a slot is free, no other request on
 * its system is running, and its neighbour list fits in hbm_budget_bytes
 * (idle systems' lists are evicted, least recently used first).  Requests on
 * one system run in submission order. */
typedef struct tmd_server tmd_server;

/* hbm_budget_bytes: device memory for system state and neighbour lists
 * (0: 32 GiB); max_slots: concurrent requests, 1..64 (0: 8); max_atoms: the
 * largest system accepted, which sizes each slot's workspace (0: 262,144);
 * skin: neighbour-list skin of MD runs (A), lists are rebuilt when an atom has
 * moved more than skin/2 since the last build; capacity: initial per-species
 * list capacity (0: from the density); batch_atoms: energy-and-force
 * requests on systems of at most this many atoms whose lists are resident are
 * served together: a slot that takes one also takes the other such requests
 * queued on idle systems (the first queued request of each system, up to 64
 * systems and max_atoms atoms) and evaluates them with one
 * tmd_energy_forces_batch call (0: off). */
typedef struct {
    int64_t hbm_budget_bytes;
    int32_t max_slots;
    int32_t device;
    int64_t max_atoms;
    double skin;
    int32_t capacity;
    int32_t batch_atoms;
} tmd_serve_opts;

typedef enum { TMD_REQ_ENERGY_FORCES = 0, TMD_REQ_MD = 1 } tmd_request_kind;

/* kind: tmd_request_kind.  MD: n_steps velocity-Verlet steps of dt_fs
 *   v += (dt/2) F/m;  x += dt v;  (rebuild the list if needed);  F = F(x);  v += (dt/2) F/m
 * with accelerations 9.648533e-3 F[eV/A]/m[amu] A/fs^2, starting from the
 * system's resident positions and either velocities (host FP64 [n][3], copied
 * at submit: for instance Maxwell-Boltzmann draws) or, when NULL, the
 * resident velocities; the final state is kept as the system's new resident
 * state.  ENERGY_FORCES evaluates the resident positions. */
typedef struct {
    int64_t system_id;
    int32_t kind;
    int32_t n_steps;
    double dt_fs;
    const double* velocities;
} tmd_request;

/* status: tmd_status of the request; energy: potential energy (MD: at the
 * final positions); kinetic: MD final kinetic energy (103.6427 * m v^2 / 2, eV);
 * virial: at the final positions; t_submit, t_start, t_done: seconds on the
 * host steady clock since the server was created; rebuilds: neighbour-list
 * builds the request made; batch_size: requests evaluated in the same launch
 * chain as this one (1: alone, 0: rejected; see batch_atoms). */
typedef struct {
    int32_t status;
    int32_t kind;
    int64_t system_id;
    int64_t n_atoms;
    int32_t n_steps;
    int32_t rebuilds;
    double energy;
    double kinetic;
    double virial[6];
    double t_submit;
    double t_start;
    double t_done;
    int32_t batch_size;
    int32_t reserved;
} tmd_result;

/* The server keeps `model` (not copied: it must outlive the server and not
 * change while requests run) and uses its precision setting. */
tmd_status tmd_serve_create(const tmd_model* model, const tmd_serve_opts* opts, tmd_server** out);
/* Register a system: host FP64 positions [n][3], host int32 species [n], box,
 * host FP64 masses per species [S] (amu).  Velocities start at zero.  When
 * hbm_budget_bytes has room, the system's neighbour list is also allocated and
 * built here (blocking the caller), so that requests on it start with a
 * resident list; otherwise, or if that build fails, its first request builds
 * it.  TMD_ERR_REJECTED when it is larger than max_atoms or its state cannot
 * fit. */
tmd_status tmd_serve_add_system(tmd_server* server, int64_t n_atoms, const double* pos, const int32_t* species,
                                const double box[3], const double* masses, int64_t* system_id);
/* Queue a request; *ticket identifies it.  Thread-safe. */
tmd_status tmd_serve_submit(tmd_server* server, const tmd_request* request, uint64_t* ticket);
/* TMD_ERR_NOT_READY until the request is done, then TMD_OK with *result
 * filled (result->status holds the request's own outcome).  Thread-safe. */
tmd_status tmd_serve_poll(tmd_server* server, uint64_t ticket, tmd_result* result);
/* Block until done (or timeout_s seconds, then TMD_ERR_NOT_READY; < 0 waits forever). */
tmd_status tmd_serve_wait(tmd_server* server, uint64_t ticket, double timeout_s, tmd_result* result);
/* Host copies of a finished request's arrays, each nullable: forces [n][3]
 * (at the final positions), pos and vel [n][3] (MD: final state), epot and
 * ekin [n_steps + 1] (MD: before the first step and after each). */
tmd_status tmd_serve_fetch(tmd_server* server, uint64_t ticket, float* forces, double* pos, double* vel,
                           double* epot, double* ekin);
/* Forget a finished request's result. */
tmd_status tmd_serve_release(tmd_server* server, uint64_t ticket);
/* Current resident positions / velocities of a system (host FP64 [n][3], nullable). */
tmd_status tmd_serve_read_system(tmd_server* server, int64_t system_id, double* pos, double* vel);
/* Device memory the server holds (system state, lists, slot workspaces) and
 * its high-water mark, in bytes. */
tmd_status tmd_serve_memory(tmd_server* server, int64_t* in_use, int64_t* peak);
/* The part of it that one system holds: its state (positions, velocities,
 * forces, species; bytes) and its neighbour list (0 while it has none resident:
 * evicted, or left to its first request).  Either pointer may be NULL;
 * TMD_ERR_INVALID_ARGUMENT for an unknown system. */
tmd_status tmd_serve_system_memory(tmd_server* server, int64_t system_id, int64_t* state_bytes, int64_t* list_bytes);
const char* tmd_serve_last_error(tmd_server* server);
/* Finish the running requests, drop queued ones, free everything. */
void tmd_serve_destroy(tmd_server* server);

#ifdef __cplusplus
}
#endif

#endif /* TMD_H */
