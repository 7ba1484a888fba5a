/*
 * itse: imaginary-time Schroedinger eigensolver on an N^3 periodic lattice,
 * MI355X (gfx950) HIP implementation.
 *
 * The method is that of arXiv:2006.16935 ("The Relativistic Schroedinger
 * Equation through FFTW 3: An Extension of quantumfdtd"):
 *
 *   psi(tau + dtau) = A psi(tau) - B dtau H_K psi(tau)          (equation iter_proced)
 *   A = (1 - dtau V/2) / (1 + dtau V/2),  B = 1 / (1 + dtau V/2) (section "The iterative procedure")
 *   H_K psi = IFFT[ T(k) FFT[psi] ] / N^3                       (equations HK1, HK2, HK3)
 *
 * with the momenta k_l = 2 pi m_l / N, m_l in (-N/2, N/2] (equation eigenmodes),
 * normalisation sum |psi|^2 = 1 over the full lattice, projection of lower
 * states and the parity projections P^(+-) psi = (psi(r) +- psi(-r))/2
 * (equation parity).
 *
 * Conventions for every entry point:
 *  - Errors: every call returns an itse_status; nothing throws across the ABI.
 *    On error, itse_last_error() returns a thread-local message.
 *  - Layout: states and potentials are real N^3 arrays in C order [x1][x2][x3]
 *    (x3 fastest).  Spectra are N x N x (N/2+1) complex, interleaved (re, im),
 *    C order [k1][k2][k3] with k3 = 0..N/2.
 *  - Memory: host pointers (on_device = 0) are read or written synchronously
 *    during the call.  Device pointers (on_device = 1) are accessed on the
 *    lattice's stream; the call returns after enqueueing unless stated.  The
 *    caller keeps ownership of every buffer it passes.  The library owns the
 *    lattice's device buffers (allocated through the optional allocator at
 *    create, released at destroy).
 *  - Asynchrony: work is enqueued on the HIP stream given at create.  Calls
 *    that return results to the host (observe, history, get_state to host,
 *    sync) synchronise that stream.
 *  - Determinism: sums are formed per workgroup and combined in a fixed order;
 *    a lattice's results do not depend on other work on the GPU or on the
 *    batch it is stepped in.
 */
#ifndef ITSE_H
#define ITSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ITSE_MAX_STATES 8

typedef enum {
    ITSE_OK = 0,
    ITSE_EINVAL = -1,      /* bad argument (size, pointer, enum, state index) */
    ITSE_ENOMEM = -2,      /* device allocation failed or over an admission budget */
    ITSE_EUNSTABLE = -3,   /* dtau * max T(k) > 1.95 or 1 + dtau min(V)/2 <= 0 */
    ITSE_ENONFINITE = -4,  /* a reduction produced NaN or Inf */
    ITSE_EDEVICE = -5,     /* a HIP runtime call failed */
    ITSE_ESTATE = -6,      /* call not valid in the object's current state */
    ITSE_ENOTFOUND = -7    /* no such request / no result yet */
} itse_status;

/* Kinetic terms (the paper's KINTERM 0..3, plus the relativistic analogue of
 * H_K^(1) the paper calls straightforward in section "Kinetic terms"). */
typedef enum {
    ITSE_KIN_FDTD = 0,     /* H_K^(0) (equation HK0): 7-point finite differences  */
                           /* / (2 A^2 M), psi = 0 outside the N^3 box (Dirichlet);*/
                           /* one stencil pass per step instead of the transforms  */
    ITSE_KIN_NR_CONT = 1,  /* H_K^(1): sum k_l^2 / (2 A^2 M)                     */
    ITSE_KIN_NR_LAT = 2,   /* H_K^(2): 4 sum sin^2(k_l/2) / (2 A^2 M)             */
    ITSE_KIN_REL_LAT = 3,  /* H_K^(3): sqrt(p^2 + M^2), p^2 = 4/A^2 sum sin^2     */
    ITSE_KIN_REL_CONT = 4  /* sqrt(p^2 + M^2), p^2 = sum k_l^2 / A^2              */
} itse_kinetic;

typedef enum {
    ITSE_FP64 = 0,         /* FP64 storage, transforms and sums                    */
    ITSE_FP32 = 1          /* FP32 storage and transforms, FP64 sums and Gram-     */
                           /* Schmidt coefficients; the kinetic symbol T(k) is    */
                           /* evaluated in FP64 and rounded once to FP32          */
} itse_precision;

typedef enum {
    ITSE_CENTER_CELL = 0,  /* potential centred at the off-grid point (N-1)/2     */
    ITSE_CENTER_ORIGIN = 1 /* potential centred at site 0 (minimum image)         */
} itse_center;

typedef enum { ITSE_DTYPE_F32 = 1, ITSE_DTYPE_F64 = 2 } itse_dtype;

/* Lattice description (the paper's NUM, A, MASS, KINTERM, EPS). */
typedef struct {
    int n;                   /* points per axis; 8..256 with prime factors 2, 3 only */
    double a;                /* lattice spacing A > 0                                 */
    double mass;             /* mass M > 0                                            */
    double dtau;             /* imaginary-time step EPS > 0                           */
    int kin;                 /* itse_kinetic                                          */
    int subtract_rest_mass;  /* relativistic forms: 1 -> sqrt(p^2+M^2) - M            */
    int precision;           /* itse_precision                                        */
    int center;              /* itse_center: coordinates of moments and mirror sites  */
    int nstates;             /* number of states evolved together, 1..ITSE_MAX_STATES */
    int complex_psi;         /* 1: one complex state (nstates must be 1) in a complex */
                             /* potential V = Re V + i Im V (itse_set_potential sets  */
                             /* Re V, itse_set_potential_imag Im V); the state is held */
                             /* as two real arrays, state index 0 = Re psi and 1 =    */
                             /* Im psi in itse_set_state / itse_get_state /           */
                             /* itse_apply_kinetic / itse_spectrum; observables under  */
                             /* index 0 only.  0: real states (zero-initialise).      */
} itse_desc;

/* Observables of one state at the start of a step (the paper's UPDATE output). */
typedef struct {
    long long step;          /* global step index of the state these describe         */
    double energy;           /* (<psi|H_K psi> + <psi|V psi>) / <psi|psi>             */
    double kinetic;          /* <psi|H_K psi> / <psi|psi>                             */
    double potential;        /* <psi|V psi> / <psi|psi>                               */
    double norm2;            /* <psi|psi>                                             */
    double x, y, z, r2;      /* <x1>, <x2>, <x3>, <r^2> about the potential centre    */
                             /* (filled when moments were requested, else 0)          */
    double parity_even;      /* weight of P^+ psi: (1 + <psi|P psi>/<psi|psi>)/2      */
                             /* (filled when moments were requested, else -1; -1 for  */
                             /* H_K^(0) lattices: itse_analyse with min_sep_edge = 0  */
                             /* gives it as w_plus)                                   */
    double energy_imag;      /* complex states: Im <psi|H psi>/<psi|psi> = <psi|Im V    */
                             /* psi>/<psi|psi> (energy, potential hold the real parts);*/
                             /* 0 for real states                                      */
} itse_obs;

/* Per-lattice step options. */
typedef struct {
    int ortho_every;                   /* Gram-Schmidt of state i against states 0..i-1  */
                                       /* after steps whose global index+1 is a multiple */
                                       /* of this; 0 = never (normalisation only)         */
    int moments;                       /* 1: also compute <x>,<y>,<z>,<r^2>, parity weight*/
    int parity[ITSE_MAX_STATES];       /* per state: 0 none, +1 / -1 reflection projection*/
    int axes[ITSE_MAX_STATES];         /* reflected axes, bit0 x1, bit1 x2, bit2 x3;      */
                                       /* 7 = inversion (P^+-), 4 / 2 = INITSYMMETRY x3/x2*/
                                       /* complex lattices: parity[0] / axes[0] project   */
                                       /* Re psi and Im psi alike; ortho_every ignored    */
} itse_step_opts;

typedef void *(*itse_alloc_fn)(size_t bytes, void *user);
typedef void (*itse_free_fn)(void *ptr, void *user);

typedef struct itse_lattice itse_lattice;
typedef struct itse_batch itse_batch;
typedef struct itse_server itse_server;

/* Thread-local message for the last failing call on this thread. */
const char *itse_last_error(void);
const char *itse_version(void);

/* Device bytes a lattice with this description holds (for admission control). */
size_t itse_footprint_bytes(const itse_desc *desc);

/* Create a lattice.  Checks n (factors 2, 3; 8..256), a, mass, dtau > 0, kin,
 * nstates, and the stability bound dtau * max_k T(k) <= 1.95 (ITSE_EUNSTABLE).
 * `hip_stream` (hipStream_t, may be NULL for the null stream) orders all work.
 * `alloc`/`free_fn` may be NULL (then hipMalloc/hipFree).  States start at 0,
 * the potential at 0, the step counter at 0. */
itse_status itse_create(const itse_desc *desc, void *hip_stream, itse_alloc_fn alloc,
                        itse_free_fn free_fn, void *alloc_user, itse_lattice **out);
itse_status itse_destroy(itse_lattice *lat);
itse_status itse_set_stream(itse_lattice *lat, void *hip_stream);

/* Potential V_b of equation iter_proced, N^3 values.  Rejects non-finite values
 * (ITSE_ENONFINITE, host input only) and 1 + dtau min(V)/2 <= 0 (ITSE_EUNSTABLE,
 * host input only; device input is checked on the device at the next step). */
itse_status itse_set_potential(itse_lattice *lat, const void *v, int dtype, int on_device);

/* Imaginary part of the potential of a complex lattice (desc.complex_psi = 1),
 * N^3 values; the step uses A = (1 - dtau V/2)/(1 + dtau V/2) and
 * B = 1/(1 + dtau V/2) with the complex V (equation iter_proced; the paper's
 * complex harmonic oscillator is such a potential).  Rejects non-finite values
 * (ITSE_ENONFINITE, host input only) and real lattices (ITSE_ESTATE). */
itse_status itse_set_potential_imag(itse_lattice *lat, const void *v, int dtype, int on_device);

/* State i (0-based), N^3 values, any normalisation (the next step normalises). */
itse_status itse_set_state(itse_lattice *lat, int i, const void *psi, int dtype, int on_device);

/* Current state i, normalised, orthogonalised as of the last step. */
itse_status itse_get_state(itse_lattice *lat, int i, void *out, int dtype, int on_device);

/* Per-lattice options used by itse_step (opts == NULL) and by batch steps. */
itse_status itse_set_step_opts(itse_lattice *lat, const itse_step_opts *opts);

/* nsteps applications of the step map to every state, each followed by the
 * optional reflection projection, then Gram-Schmidt / normalisation
 * (order: update, projection, Gram-Schmidt in state order, normalise).
 * Observables of each state at the start of each step are recorded.  A complex
 * lattice takes the map with complex A and B, the projection of both parts and
 * the normalisation sum |Re psi|^2 + |Im psi|^2 = 1; it records one observable
 * per step (index 0) with energy_imag. */
itse_status itse_step(itse_lattice *lat, int nsteps, const itse_step_opts *opts);

/* Observables of the current states without stepping (no update). */
itse_status itse_evaluate(itse_lattice *lat, int moments);

/* Latest observables of state i (from the last step or evaluate).  Synchronises. */
itse_status itse_observe(itse_lattice *lat, int i, itse_obs *out);

/* Observables of the last `count` steps (oldest first), count <= 4096 and
 * <= steps taken; out holds count * nstates records.  Synchronises. */
itse_status itse_history(itse_lattice *lat, int count, itse_obs *out);

long long itse_step_count(const itse_lattice *lat);

/* Entry points for real states only (ITSE_ESTATE on a complex lattice):
 * itse_orthogonalise, itse_project_parity, itse_polish, itse_analyse,
 * itse_momentum_radial, itse_snapshot_push, itse_snapshot_extract; and the
 * server takes real states only. */

/* Modified Gram-Schmidt of state i against states 0..i-1, then normalise: the
 * removal of the components along the lower states by which excited states are
 * extracted, and the full-volume normalisation sum |psi|^2 = 1 (section "The
 * iterative procedure").  Errors: ITSE_EINVAL (index), ITSE_ENONFINITE (state i in
 * the span of the lower states), ITSE_ESTATE (complex lattice).  Synchronises. */
itse_status itse_orthogonalise(itse_lattice *lat, int i);

/* P psi_i = (psi_i + sign * psi_i o R)/2 with R reflecting `axes`, then
 * normalise; *weight (optional) receives ||P psi||^2 / ||psi||^2.  Synchronises. */
itse_status itse_project_parity(itse_lattice *lat, int i, int sign, int axes, double *weight);

/* H_K psi_i written to `out_device` (N^3 values in the lattice precision). */
itse_status itse_apply_kinetic(itse_lattice *lat, int i, void *out_device);

/* Unnormalised forward transform FFT[psi_i], half spectrum N x N x (N/2+1)
 * complex in the lattice precision, written to `out_device`. */
itse_status itse_spectrum(itse_lattice *lat, int i, void *out_device);

/* FP64 re-evaluation of state i's observables with an FP64 kinetic application
 * (for FP32 lattices: the energy of the FP32 state without FP32 transform error).
 * Synchronises. */
itse_status itse_polish(itse_lattice *lat, int i, itse_obs *out);

/* ---- Analysis of a state -------------------------------------------------
 * Box normalisation and average radius (section "Finite volume normalization")
 * and parity weights (section "Parity projection") in the effective volume: the
 * sites whose coordinates about the potential centre all satisfy
 * |c_l| <= (1 - min_sep_edge) N A / 2 (a box of side (1 - min_sep_edge) A N). */
typedef struct {
    double box_norm2;        /* sum over the box of psi^2 (psi as held: unit norm on the lattice) */
    double rho_box;          /* <rho> in the box after box normalisation, lattice units */
    double w_plus, w_minus;  /* box weights of P+ and P- (full inversion)              */
    double w_minus_axis[3];  /* box weights of P-_{e_k} = (1 + R_perp)(1 - R_k)/4       */
} itse_analysis;

/* Analysis of state i, 0 <= min_sep_edge < 1.  FP64 sums in a fixed order.  The
 * first call allocates a few KiB of partial sums through the lattice's allocator.
 * Synchronises.  Errors: ITSE_EINVAL, ITSE_ENONFINITE if the box holds no weight. */
itse_status itse_analyse(itse_lattice *lat, int i, double min_sep_edge, itse_analysis *out);

/* itse_analyse for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the partial sums in a fixed workspace the library
 * holds on each GPU it runs on (112 KiB per GPU, held until the process ends; it
 * covers every supported n, and a larger need is refused with ITSE_EINVAL).  No
 * device memory is allocated or freed by the call.  The workspace is shared by
 * all calls on one GPU: calls that overlap on the same GPU (from several
 * threads or on several streams) race, and the caller must order them.
 * Synchronises the lattice's stream.  Errors as for itse_analyse, and
 * ITSE_EDEVICE if the workspace's address cannot be obtained. */
itse_status itse_analyse_noalloc(itse_lattice *lat, int i, double min_sep_edge, itse_analysis *out);

/* Radial momentum-space wave-function of state i: Psi(p) = FFT[psi] scaled so that
 * (2 pi / (N A))^3 sum_p |Psi(p)|^2 = 1, p on the eigenmode set; momenta grouped in
 * bins of width 2 pi / (N A) (bin b: |p| in [(b - 1/2), (b + 1/2)) 2 pi / (N A)),
 * b < nbins <= 512.  Per bin: count[b] momenta, their mean |p| in p[b], the mean
 * |Psi(p)| in psi[b] and y[b] = sqrt(4 pi) p[b] psi[b] (0 for empty bins).  Any of
 * the output arrays may be NULL.  The first call allocates a half spectrum and the
 * partial histograms through the lattice's allocator.  Histogram sums use LDS
 * atomics (their order within a workgroup is the hardware's).  Synchronises. */
itse_status itse_momentum_radial(itse_lattice *lat, int i, int nbins, double *count, double *p, double *psi,
                                 double *y);

/* ---- Snapshot-overlap extraction of excited states ----------------------
 * The paper's procedure (section "The iterative procedure"): while state 0
 * evolves, snapshots of it are kept; the latest wave-function estimates the
 * ground state, and each earlier snapshot, newest first, with its projections
 * on the estimates found so far removed and then normalised, estimates the next
 * state.  The library keeps the ITSE_SNAPSHOTS latest snapshots of state 0. */
#define ITSE_SNAPSHOTS 2

/* Copies the current state 0 into the snapshot ring; when the ring is full the
 * oldest snapshot is dropped.  The first call allocates the ring (ITSE_SNAPSHOTS
 * arrays of N^3 values in the lattice precision, through the lattice's
 * allocator; not part of itse_footprint_bytes).  Asynchronous on the lattice
 * stream.  Errors: ITSE_ENOMEM. */
itse_status itse_snapshot_push(itse_lattice *lat);

/* Number of snapshots held, 0..ITSE_SNAPSHOTS. */
itse_status itse_snapshot_count(const itse_lattice *lat, int *count);

/* Drops the snapshots (the ring stays allocated). */
itse_status itse_snapshot_clear(itse_lattice *lat);

/* Forms the 1 + count estimates from the current state 0 and the snapshots and
 * writes their observables (FP64 Rayleigh quotients, norms, moments, parity
 * weights) to out[0 .. 1 + count); *n_out receives 1 + count.  If states_out is
 * not NULL, estimate e is written at states_out + e N^3 values of `dtype`
 * (ITSE_DTYPE_F32 or ITSE_DTYPE_F64), in host or device memory per on_device.
 * The lattice's own states and snapshots are not changed.  Synchronises.
 * Errors: ITSE_ENONFINITE if a snapshot lies in the span of the later ones. */
itse_status itse_snapshot_extract(itse_lattice *lat, itse_obs *out, int *n_out, void *states_out, int dtype,
                                  int on_device);

/* Per-pass timing: `nsteps` steps launched eagerly with HIP events recorded
 * between consecutive kernel launches on the lattice stream.  On input *npass is
 * the capacity of ms_out; on output the number of passes per step, with
 * ms_out[p] the mean duration of pass p.  `names` (optional) receives a JSON
 * array of the pass kernel names.  The steps are real steps (the state advances).
 * Synchronises. */
itse_status itse_profile_step(itse_lattice *lat, int nsteps, double *ms_out, int *npass, char *names,
                              size_t names_len);

/* Wait for all work enqueued for the lattice; reports device-side errors. */
itse_status itse_sync(itse_lattice *lat);

/* ---- batched stepping: independent lattices stepped together ------------------ */
/* Lattices of equal (n, precision) share each pass's launch; the whole chunk of
 * steps for all lattices is captured once into a HIP graph and replayed.  A
 * lattice's results are bitwise identical to stepping it alone. */
itse_status itse_batch_create(int count, itse_lattice *const *lats, void *hip_stream,
                              itse_batch **out);
itse_status itse_batch_step(itse_batch *b, int nsteps);
itse_status itse_batch_destroy(itse_batch *b);
/* Persistent stepping (on = 1): each itse_batch_step is then one cooperative launch
 * of a kernel whose resident workgroups run the passes of every lattice of the
 * batch for all the steps, the passes separated by grid-wide barriers (the tiles
 * are those of the passes' own kernels, so results stay bitwise those of each
 * lattice stepped alone).  Takes FP32 transform lattices of real states with N in
 * {32, 48, 64, 96} created under a schedule variant whose plane and column
 * workgroups have 256 threads (1 at each of these N, 2 at N = 48, 64 and 96), at
 * most two states, in at most eight groups of equal (N, schedule); otherwise
 * ITSE_EINVAL.  Steps whose options need position moments or projections of
 * states along different axes take the graph path.  on = 0
 * returns to graph replay (the default, and the faster path on MI355X: each
 * grid-wide barrier there costs tens of microseconds, several per step). */
itse_status itse_batch_set_persistent(itse_batch *b, int on);

/* ---- schedules ------------------------------------------------------------------ */
/* Schedules are kept per (n, precision) and per kind of lattice: one state, or
 * several (their best schedules differ).  A lattice takes the schedule current at
 * its creation.  Results stay deterministic for a given schedule. */
/* Time the available transform schedules for (n, precision) on the current
 * device, on a three-state step (parity +, -, -, Gram-Schmidt) and on a bare
 * one-state step, and keep the fastest of each for later lattices of that shape.
 * `json` (optional) receives the timings ("times_ms", "times_ms_one_state") and
 * the choices ("best", "best_one_state"). */
itse_status itse_autotune(int n, int precision, void *hip_stream, char *json, size_t json_len);
/* The same for lattices stepped together: times a batch of `count` lattices of
 * (n, precision) with `nstates` states each (Gram-Schmidt every step) under every
 * schedule and keeps the fastest for that kind of lattice (several states, or one)
 * -- with many lattices in a batch there is parallelism enough without finer
 * splits, so the choice can differ from itse_autotune's.  `json` receives
 * "times_ms" (per step of the batch) and "best".  Allocates and frees the
 * lattices it times (about count times one lattice's footprint); errors:
 * ITSE_EINVAL (count < 1, nstates outside 1..ITSE_MAX_STATES, unknown shape),
 * ITSE_ENOMEM, ITSE_EDEVICE. */
itse_status itse_autotune_batch(int n, int precision, int count, int nstates, void *hip_stream, char *json,
                                size_t json_len);
/* Description of the current multi-state schedule, with "variant_one_state". */
itse_status itse_schedule_get(int n, int precision, char *json, size_t json_len);
/* Set the schedule of both kinds of lattice; errors: ITSE_EINVAL for an unknown
 * (n, precision) or variant. */
itse_status itse_schedule_set(int n, int precision, int variant);
/* Set the schedule of lattices with `nstates` states (1: one-state lattices,
 * 2..ITSE_MAX_STATES: the multi-state ones). */
itse_status itse_schedule_set_states(int n, int precision, int nstates, int variant);

/* ---- serving: eigensolve requests with admission by HBM footprint ---------------- */
/* A server owns the lattices of the requests it has admitted.  Requests wait in
 * arrival order until their footprint (itse_footprint_bytes) fits the server's
 * HBM budget beside the admitted ones and a slot is free; admitted requests are
 * stepped together (continuous batching: all live lattices advance by one chunk
 * of steps per itse_server_progress call, each in its own arrays, so a request's
 * results do not depend on what else is live).  After every chunk each request
 * compares its energies with those one chunk earlier (the paper's tolerance test,
 * section "Basic configuration", on |dE|) and completes when every state moved by
 * at most tol (relative to |E| when tol_relative), or at max_steps.  The calls are
 * not thread-safe: one host thread drives a server. */
typedef struct {
    itse_desc desc;              /* lattice, kinetic term, precision, states          */
    const void *potential;       /* host, N^3 values of potential_dtype               */
    int potential_dtype;         /* itse_dtype                                        */
    const void *const *states;   /* host, desc.nstates arrays of state_dtype          */
    int state_dtype;             /* itse_dtype                                        */
    itse_step_opts opts;         /* projections and Gram-Schmidt interval             */
    double tol;                  /* energy change per chunk that counts as converged  */
    int tol_relative;            /* 1: tol relative to |E|                            */
    int keep_states;             /* 1: keep the final states for itse_server_state    */
    long long max_steps;         /* give up after this many steps (converged = 0)     */
} itse_request;

typedef struct {
    uint64_t id;                 /* as returned by itse_server_submit                 */
    int status;                  /* itse_status of the solve                          */
    int converged;               /* 1 if the tolerance was met                        */
    long long steps;             /* steps taken                                       */
    double energy[ITSE_MAX_STATES];  /* final energies (FP64 sums)                   */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock               */
} itse_result;

/* hbm_budget: device bytes the admitted lattices may hold in total; max_slots:
 * most requests live at once; chunk: steps per itse_server_progress.  Work runs
 * on hip_stream (may be NULL). */
itse_status itse_server_create(size_t hbm_budget, int max_slots, int chunk, void *hip_stream,
                               itse_server **out);
itse_status itse_server_destroy(itse_server *s);
/* Copies the request's host arrays (they may be freed on return).  Rejects a
 * request whose footprint alone exceeds the budget (ITSE_ENOMEM) and invalid
 * descriptions (ITSE_EINVAL, ITSE_EUNSTABLE) at once. */
itse_status itse_server_submit(itse_server *s, const itse_request *req, uint64_t *id);
/* Admit what fits, step every live request by one chunk, test convergence,
 * retire finished requests (freeing their device memory).  *live and *queued
 * (optional) receive the counts after the call.  Synchronises the stream. */
itse_status itse_server_progress(itse_server *s, int *live, int *queued);
/* Up to max finished results, oldest first; *n_out receives the count. */
itse_status itse_server_poll(itse_server *s, itse_result *out, int max, int *n_out);
/* Final state i of a finished request submitted with keep_states, as N^3 values of
 * dtype into host memory; itse_server_release drops the kept states. */
itse_status itse_server_state(itse_server *s, uint64_t id, int i, void *out, int dtype);
itse_status itse_server_release(itse_server *s, uint64_t id);
/* Device bytes currently held by admitted requests. */
size_t itse_server_bytes_in_use(const itse_server *s);

#ifdef __cplusplus
}
#endif

#endif /* ITSE_H */
