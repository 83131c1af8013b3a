/*
 * libusp: MI355X (gfx950) particle solver for the unified stochastic particle
 * ES-BGK method (USP-ESBGK) of Fei, Zhang, Li and Liu, "A Unified Stochastic
 * Particle Bhatnagar-Gross-Krook Method for Multiscale Gas Flows"
 * (arXiv 1808.03801).
 *
 * One call of usp_step advances every listed instance by the per-time-step
 * algorithm of Table 2 (steps 2-8): added particles for f-hat^n (Eq. 22,
 * 25-26), advection with wall reflection, a stable counting sort by cell,
 * the moments of f-tilde^* and the starred stress / heat flux (Eq. 33),
 * added particles for f^* (Eq. 24), Bernoulli selection and reassignment
 * (Eq. 9, 28), resampling from the time-dependent ES Gaussian (Eq. 6, 29-32),
 * added particles for the last term of Eq. 27, a per-cell conservation
 * correction, the moments of f^{n+1} (Eq. 1), their time average (Eq. 34) and
 * P_ne (Eq. 16-18).  All of it runs in HIP kernels on the device.
 *
 * Conventions
 *  - Every function returns a usp_status; 0 is success.  The text of the last
 *    error of a context is returned by usp_last_error.
 *  - Argument errors are reported synchronously.  Errors raised inside the
 *    kernels (capacity, window, non-finite moments) are sticky per instance
 *    and reported by the next usp_sync / usp_get_* call on it; a failed
 *    instance refuses further steps with USP_ESTATE, other instances
 *    continue.
 *  - The context owns all device memory it allocates (through the caller's
 *    allocator if one is given).  The caller owns every host buffer passed in.
 *  - All work is enqueued on the context's HIP stream; usp_step returns
 *    without waiting.
 *  - 1-D problems resolve y only; 2-D problems resolve x and y; velocities
 *    always have three components; cells are numbered iy * nx + ix.
 *  - Host particle records are [x, y, cx, cy, cz, w] doubles in canonical
 *    order (cell by cell; within a cell the order the algorithm defines).
 */
#ifndef USP_H
#define USP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    USP_OK = 0,
    USP_EINVAL = -1,    /* bad argument or configuration */
    USP_ENOMEM = -2,    /* device allocation failed / footprint above budget */
    USP_ECAPACITY = -3, /* a cell exceeded max_ppc particles (instance poisoned) */
    USP_EWINDOW = -4,   /* a particle moved farther than the sort window (poisoned) */
    USP_EDEVICE = -5,   /* a HIP runtime call failed */
    USP_ESTATE = -7,    /* instance unknown, freed or poisoned */
    USP_ENOLIB = -8,    /* built without device support */
    USP_ENONFINITE = -9 /* a cell moment became infinite or NaN (instance poisoned) */
} usp_status;

enum { USP_BC_DIFFUSE = 0, USP_BC_SPECULAR = 1, USP_BC_PERIODIC = 2, USP_BC_OPEN = 3 };
enum { USP_PNE_FIXED = 0, USP_PNE_GLL_INST = 1, USP_PNE_GLL_AVG = 2 };
enum { USP_WEIGHT_CONSISTENT = 0, USP_WEIGHT_LITERAL = 1 };
enum { USP_CONSERVE_FULL = 0, USP_CONSERVE_NONE = 1 };
enum { USP_JMOM_INST = 0, USP_JMOM_AVG = 1 };
enum { USP_SCHEME_USP = 0, USP_SCHEME_SP = 1 };
enum { USP_ES_SAMPLED = 0, USP_ES_MEAN = 1 };
enum { USP_GLL_U_SOUND = 0, USP_GLL_U_LITERAL = 1 };
enum { USP_SELECT_BERNOULLI = 0, USP_SELECT_COUNT = 1 };
enum { USP_ES_SAMPLER_CHOLESKY = 0, USP_ES_SAMPLER_LINEAR = 1 };

/* Gas (Section 4): Eq. 35 viscosity mu = mu_ref (T / T_ref)^omega; Pr of
 * Eq. 6 (nu_ES = Pr nu); molecular mass m and Boltzmann constant kB. */
typedef struct {
    double m, kB, mu_ref, T_ref, omega, Pr;
} usp_gas;

/* A face of the domain: kind USP_BC_*, wall temperature T and wall velocity u
 * (diffuse faces; full accommodation).
 *
 * Open faces (USP_BC_OPEN; the Sod tube's open ends of Section 4.3 and the
 * reservoirs of the slit of Section 4.5): the face borders a reservoir of gas
 * with number density n (1/m^3), temperature T and velocity u, whose
 * component normal to the face must be 0.  A particle that reaches the face
 * leaves the domain; every step, the reservoir's molecules that cross the
 * face enter: per boundary cell a stochastically rounded n sqrt(kT/(2 pi m))
 * A dt / Np of them (A = the cell's share of the face: unit area in 1-D, dx or
 * dy per unit depth in 2-D), each at a uniform point of that share and a
 * uniform time of the step, with a velocity from the flux-weighted half-range
 * Maxwellian, weight 1.  On the part of a face whose tangential coordinate
 * (2-D: x on a y face, y on an x face; the cell centre decides) is >= split,
 * the reservoir has density n_b and temperature T_b instead (a face that
 * borders two chambers); split = +inf for a uniform face.  Open faces cannot
 * be combined with a body acceleration. */
typedef struct {
    int kind;
    double T;
    double u[3];
    double n, split, n_b, T_b;
} usp_face;

/* Geometry.  Domain [x0, x1] x [y0, y1] with nx * ny uniform cells of widths
 * dx, dy (inv_dx = 1/dx, inv_dy = 1/dy supplied so that every solver uses the
 * same numbers); vcell = cell volume (per unit depth / area in 2-D / 1-D).
 * face[0..3] = x-lo, x-hi, y-lo, y-hi (x faces are unused in 1-D; a periodic
 * face needs a periodic opposite face).  accel = uniform body acceleration
 * (the Poiseuille drive), m/s^2.  plate != 0 (2-D only): a thin diffuse wall
 * at rest and at temperature plate_T on the line x = plate_x (strictly inside
 * the domain) for plate_ylo <= y <= plate_yhi, reflecting on both sides (the
 * wall between the two chambers of the slit, Section 4.5). */
typedef struct {
    int dim, nx, ny;
    double x0, x1, y0, y1, dx, dy, inv_dx, inv_dy, vcell;
    usp_face face[4];
    double accel[3];
    int plate;
    double plate_x, plate_ylo, plate_yhi, plate_T;
} usp_problem;

/* Numerics.  dt: time step (s); Np: real molecules per unit weight; r_p:
 * Eq. 25 scale (10 in the paper); Kn_c: Eq. 16 reference Knudsen number
 * (0.1); pne_mode: USP_PNE_*, pne_fixed used by USP_PNE_FIXED; n_avg: Eq. 34
 * window (1000) and avg_start: first averaged step; precision: 32 or 64
 * (particle state); max_ppc: largest number of particles a cell may hold
 * during a step (<= 2048; <= 1365 for a problem with open faces or the
 * plate, else usp_create fails with USP_EINVAL); jmom_mode: moments that build the added particles
 * and the ES target (instantaneous Eq. 1 or averaged Eq. 34);
 * spawn_projection: 1 = project each added batch onto zero mass, momentum and
 * energy; window: sort-window half width in cells (0 = derive from the
 * initial state); avg_init: start of the Eq. 34 averages (both the averaged
 * fields and the averages of f-tilde^* that jmom_mode uses): 0 = the first
 * sample, then a running mean until n_avg samples; 1 = the exact raw moments
 * of the initial Maxwellian state, then the fixed window n_avg.
 * scheme: USP_SCHEME_USP (Table 2, the default) or USP_SCHEME_SP, the
 * SP-ESBGK baseline of Table 1: no added particles (requires pne_mode
 * USP_PNE_FIXED with pne_fixed = 0), the Eq. 9 count of particles (nearest
 * integer of N_c (1 - exp(-nu_ES dt)), the smallest rank keys of the cell)
 * reassigned and none deleted, their velocities a Maxwellian thermal
 * velocity mapped by Eq. 11 (S = I - (1 - Pr) / (2 Pr) sigma / p) around the
 * cell's velocity; the conservation correction as for USP.
 * es_mode: USP_ES_SAMPLED (the paper: each reassigned particle of step 6
 * draws a time t from Eq. 29-30 and takes f_G with alpha(t) of Eq. 32) or
 * USP_ES_MEAN: alpha replaced by its expectation over that time distribution,
 * P + (1 - P) Pr (e^{(Pr - 1) nu dt} - 1) / ((Pr - 1)(e^{Pr nu dt} - 1)), one
 * Gaussian per cell with the same second moments (Pr != 1 required).
 * gll_u: the velocity term of Eq. 18, lambda |grad |u|| / Q: USP_GLL_U_SOUND
 * (Q = max(|u|, sqrt(5 theta / 3)), the convention of the GLL criterion's
 * authors; finite at stagnation) or USP_GLL_U_LITERAL (Q = |u| as printed;
 * a cell at rest with a velocity gradient gets P_ne = 0).
 * select_mode: step 5 of USP-ESBGK: USP_SELECT_BERNOULLI (each particle
 * selected with probability 1 - exp(-nu_ES dt), the rate of Eq. 9) or
 * USP_SELECT_COUNT (Eq. 9 as printed: N_s = nearest(N_c (1 - exp(-nu_ES
 * dt))) particles of the cell, the ones with the smallest rank keys, are
 * the selected ones; Eq. 28 then keeps int(sum of their weights)).
 * es_sampler: step 6 sampler of f_G(t) (Eq. 32): USP_ES_SAMPLER_CHOLESKY
 * (u + L z with L the Cholesky factor of its covariance theta I + (1 - 1/Pr)
 * alpha sigma / rho, exact) or USP_ES_SAMPLER_LINEAR (the linear map of
 * Eq. 10-11 with alpha sigma in place of sigma: u + sqrt(theta) S z, S = I -
 * (1 - Pr) / (2 Pr) alpha sigma / p; covariance exact to first order in
 * sigma / p, its trace above the target's by theta ((1 - Pr) / (2 Pr))^2
 * alpha^2 tr((sigma / p)^2); theta S S^T is never indefinite, so no
 * reassignment takes the isotropic fallback of the Cholesky sampler).
 * Applies to USP_SCHEME_USP; the SP-ESBGK scheme always uses the map. */
typedef struct {
    double dt, Np, r_p, Kn_c, pne_fixed;
    int pne_mode, n_avg, avg_start, precision, weight_mode, conserve_mode, max_ppc;
    int jmom_mode, spawn_projection, window;
    uint64_t seed;
    int avg_init;
    int scheme;
    int es_mode;
    int gll_u;
    int select_mode;
    int es_sampler;
} usp_numerics;

/* Device binding.  alloc/free: device allocator (NULL = hipMalloc/hipFree);
 * user: passed back to them; stream: hipStream_t (NULL = null stream);
 * device: HIP device ordinal; budget: bytes the context may allocate
 * (0 = unlimited). */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
    void* stream;
    int device;
    size_t budget;
} usp_device;

typedef struct usp_ctx usp_ctx;

/* Creates a context bound to one device and stream. */
usp_status usp_create(const usp_device* dev, usp_ctx** out);
/* Frees every instance and the context. */
void usp_destroy(usp_ctx* ctx);
/* Text of the last error of ctx (never NULL). */
const char* usp_last_error(usp_ctx* ctx);

/* Device bytes an instance of this problem needs (admission control). */
usp_status usp_footprint(const usp_problem* pb, const usp_numerics* nm, size_t* bytes_out);

/* Creates an instance and its initial state (Table 2 step 1): per cell
 * round(n V / Np) particles, uniform positions, Maxwellian velocities at the
 * cell's (u, T), weight 1; then the moments of f^0 and P_ne^0.  init_n [ncell]
 * (1/m^3), init_u [ncell][3] (m/s), init_T [ncell] (K) are host arrays.
 * Refused with USP_EINVAL: an invalid argument or mode value, more than 2^26
 * cells, cells x capacity (max_ppc rounded up to 64) of 2^31 particle slots
 * or more (a slot of the instance is addressed by 31 bits), or an open face
 * whose reservoir would bring more than max_ppc particles into a boundary
 * cell per step on average (n sqrt(kB T / (2 pi m)) area dt / Np), or an
 * initial field that is not finite, a negative density or temperature.  A
 * cell whose initial count exceeds max_ppc sets the sticky USP_ECAPACITY. */
usp_status usp_instance_init(usp_ctx* ctx, const usp_gas* gas, const usp_problem* pb,
                             const usp_numerics* nm, const double* init_n,
                             const double* init_u, const double* init_T, int* id_out);
usp_status usp_instance_free(usp_ctx* ctx, int id);

/* Advances the n_ids listed instances by nsteps time steps each (Table 2
 * steps 2-8 per step).  Instances of one kernel flavour (state precision,
 * dimension, launch shape) share every kernel launch (batched); flavours run
 * side by side on internal streams forked from and joined back to the
 * context's stream.  Asynchronous: returns once the work is enqueued.
 * Errors: USP_EINVAL (no ids, or an id listed twice), USP_ESTATE (unknown,
 * freed or failed id), USP_ENOMEM (batch tables), USP_EDEVICE (HIP launch or
 * capture failure). */
usp_status usp_step(usp_ctx* ctx, const int* ids, int n_ids, int nsteps);

/* usp_step for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it.  Same arguments and the same results, bit for bit, as usp_step;
 * the instances themselves are created beforehand (usp_instance_init
 * allocates).  The call allocates nothing: the batch descriptor table, the
 * per-group base offsets and the shape-tier lists live in a static device
 * array of about 15 MiB that the library holds on each device it runs on
 * until the process ends.  Flavour groups run one after another on the
 * context's stream (no internal streams, no graph, no timing events; kernel
 * timing is not recorded for these calls).  Limits: at most 1024 instances
 * and 524288 cells in one call, else USP_EINVAL before anything is enqueued.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (from several contexts or host threads, or on streams not
 * ordered with each other) race and must not be made.  Errors: as usp_step,
 * plus USP_EINVAL for the limits and USP_EDEVICE when the array's address
 * could not be taken at usp_create. */
usp_status usp_step_noalloc(usp_ctx* ctx, const int* ids, int n_ids, int nsteps);

/* Waits for the stream; reports the first sticky instance error, if any. */
usp_status usp_sync(usp_ctx* ctx);
/* Sticky device error status of one instance (synchronises). */
usp_status usp_instance_status(usp_ctx* ctx, int id);

/* Number of cells / particles (synchronises). */
usp_status usp_num_cells(usp_ctx* ctx, int id, int* ncell);
usp_status usp_num_particles(usp_ctx* ctx, int id, long long* n);

/* State transfer (synchronises).  counts [ncell]; parts [N][6]; cells
 * [ncell][54] = centred moments (S0, u[3], K[6], Q[3]), raw sums (S0, S1[3],
 * S2[6], S3[3]), time-averaged raw sums of f^n, of f-tilde^*, P_ne^n,
 * P_ne^{n-1}.  get: parts may be NULL (counts only).  set: cells may be NULL
 * (moments recomputed, averages cleared, P_ne from the fields); step and
 * n_samples must be non-negative (USP_EINVAL) and every count within
 * [0, max_ppc] (USP_ECAPACITY). */
usp_status usp_get_state(usp_ctx* ctx, int id, int* counts, double* parts, double* cells,
                         int* step, int* n_samples);
usp_status usp_set_state(usp_ctx* ctx, int id, const int* counts, const double* parts,
                         const double* cells, int step, int n_samples);

/* Field record per cell (which = 0 instantaneous, 1 time-averaged), [ncell][18]:
 * S0, rho, u[3], T, p, sigma[6] (xx yy zz xy xz yz), q[3], P_ne, count. */
usp_status usp_get_fields(usp_ctx* ctx, int id, int which, double* out);

/* The same field record on the device, borrowed (no copy, no
 * synchronisation): the fields are computed on the context's stream into a
 * buffer of the instance, field-major: data[k * ncell + c] for field k of
 * cell c, k as in usp_get_fields (nfield = 18).  The buffer belongs to the
 * instance (allocated on first use, freed with it); its contents stay valid
 * until the next usp_step, usp_set_state, usp_moments or usp_instance_free
 * of the instance.  USP_EINVAL for a bad id, which or out; USP_ENOMEM when
 * the buffer cannot be allocated. */
typedef struct {
    int ncell, nfield;
    const double* data;
} usp_moments_view;
usp_status usp_moments(usp_ctx* ctx, int id, int which, usp_moments_view* out);

/* Per-cell diagnostics, [ncell][48] (enable first with usp_set_diag; costs a
 * few record writes per cell per step).  Slots 0..31 describe the last step
 * (same meaning as the oracle's record; slot 10 is a bit set: 1 invalid
 * moments, no relaxation; 2 mass correction failed; 4 momentum / energy
 * correction failed; 8 nothing reassigned; 16 whole-cell correction made);
 * slots 32..46 accumulate the shader
 * cycles spent in each phase of the cell kernel (gather, moments, step 4,
 * selection, rank selection, resampling, step 7, conservation, compaction,
 * step-8 moments, step 2, advection, bin counts, bin offsets, writes). */
usp_status usp_set_diag(usp_ctx* ctx, int id, int on);
usp_status usp_get_diag(usp_ctx* ctx, int id, double* out);

/* The stable counting sort of the last time step's step 3 (Table 2: the
 * particles sorted into cells after advection, "similar to DSMC"): the
 * particles of f-tilde^* that Eq. 33 sums, cell by cell, each cell in
 * canonical order (source offset in the sort window, then source slot).
 * cell_offsets [ncell + 1]: first sorted particle of each cell
 * (cell_offsets[ncell] = N).  perm [N] (may be NULL, to learn N first): for
 * each sorted particle its place in the sequence before the sort, which
 * lists the cells in order and, per cell, its particles of f^n in canonical
 * order, then its step-2 particles, then the particles that entered through
 * its open faces (those that left through an open face keep their place).
 * Valid after a usp_step call made with diagnostics on (usp_set_diag; the
 * record is kept in its buffers); USP_ESTATE otherwise or after
 * usp_set_state.  Host arrays, owned by the caller; synchronises. */
usp_status usp_get_sort(usp_ctx* ctx, int id, int32_t* cell_offsets, int32_t* perm);

/* Counters of one instance (synchronises).  live, step and error always;
 * diag = 1 when the rest describes the last time step (a usp_step call made
 * with diagnostics on), else 0 and the rest is zero.  added: particles of
 * the Eq. 25 batches of steps 2, 4 and 7; selected / reassigned / deleted:
 * step 5 (Eq. 9, 28); entered / left: through open faces; clamped: wall
 * traces stopped after 16 hits; es_fallback: step-6 Gaussians whose FP64
 * Cholesky factor fell back to theta I; cells_invalid: cells with fewer than
 * two particles or no positive mass or temperature (not relaxed);
 * mass_fail / energy_fail: cells whose conservation correction was skipped;
 * whole_cell: cells corrected by the whole-cell shift and scale. */
typedef struct {
    long long live;
    int step;
    int error;
    int diag;
    long long added[3];
    long long selected, reassigned, deleted;
    long long entered, left, clamped, es_fallback;
    long long cells_invalid, mass_fail, energy_fail, whole_cell;
} usp_stats_t;
usp_status usp_stats(usp_ctx* ctx, int id, usp_stats_t* out);

/* Launch shape: threads per cell workgroup.  The cell kernel keeps a cell's
 * particles in the registers of 256 threads, so 256 (or 0 for the default)
 * is the only accepted value; others return USP_EINVAL. */
usp_status usp_set_block(usp_ctx* ctx, int threads);

/* Launch shapes of the cell kernel.  Workgroup shapes s = 0..4 hold a cell
 * in 256 threads x {1, 2, 4, 4|6, 8}[s] particle slots per thread (4|6: the
 * cell reruns with 6 slots when 4 are too few); wave shapes 5 and 6 hold a
 * cell in one 64-lane wave with 4 and 6 slots per lane (shape 6 only for
 * instances without open faces or the plate).  An instance's last shape is
 * the smallest workgroup shape that holds max_ppc.  Its first shape runs
 * every cell; cells that need more slots are handed on, before anything of
 * them is written, to the workgroup shapes with more slots, up to the last.
 * The default first shape is a wave shape when the initial particles per
 * cell leave room for the added particles in one wave (4 or 6 slots), else
 * the smaller of the last shape and shape 3.  Shapes of one family
 * (workgroup or wave) reduce in the same order and give bit-identical
 * results; the two families reduce in different orders, so moving an
 * instance to the other family changes the last bits of its moments (every
 * shape passes the same parity bar).  usp_set_shape is the knob an
 * autotuner turns; first = -1 restores the default.  Errors: USP_ESTATE
 * (unknown id), USP_EINVAL (a workgroup shape above the last, a value
 * outside [-1, nshape), or shape 6 for an instance with open faces or the
 * plate).  usp_get_shape returns the first and last shape in use and the
 * number of shapes (7). */
usp_status usp_set_shape(usp_ctx* ctx, int id, int first);
usp_status usp_get_shape(usp_ctx* ctx, int id, int* first, int* last, int* nshape);

/* Graph replay (the fused, batched step captured once).
 * While on, the first usp_step call for a given list of instances and step
 * count is captured into a HIP graph (kernels only: no memory set or copy is
 * recorded) and launched; later calls with the same ids and nsteps replay
 * that graph on the context's stream.  Results are bit-identical to eager
 * launches.  Graphs are dropped when an instance is created or freed.
 * Timing mode (below) launches eagerly.  Returns USP_EINVAL for a null ctx. */
usp_status usp_set_graph(usp_ctx* ctx, int on);

/* Kernel timing (benchmarking): while on, every pass of the fused cell
 * kernel (the launches of all shapes over the cells of one step) is
 * bracketed by two HIP events on the stream it runs on; the stream is
 * drained before each pass, so that the pass's launches are queued behind
 * its start event at once.  Timing mode launches eagerly (no graphs).
 * usp_get_timing synchronises and returns the summed event time of those
 * passes (ms) and their number since timing was switched on. */
usp_status usp_set_timing(usp_ctx* ctx, int on);
usp_status usp_get_timing(usp_ctx* ctx, double* ms, long long* passes);

/* Philox4x32-10 evaluated on the device for n counters (ctr [n][4], out
 * [n][4], host arrays) with key (k0, k1); for checking the generator. */
usp_status usp_philox(usp_ctx* ctx, const uint32_t* ctr, uint32_t k0, uint32_t k1, int n,
                      uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif
