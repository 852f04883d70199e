/*
 * avl.h -- C ABI of libavl, an MI355X (gfx950) implementation of one time step
 * of the Vlasov-hybrid simulation (VHS) method of Kilian, Schreiner & Spanier,
 * "Afterlive" (arXiv:1804.03901), for one spatial and one or three velocity
 * dimensions, electrostatic, one kinetic species over an immobile neutralising
 * background.
 *
 * The step (Sec. 2, Fig. "algorithm"): markers move along the characteristics
 * of the Vlasov equation (Eq. (vlasov)) in the self-consistent field; the
 * phase-space density is rebuilt on the Eulerian grid by the weight-normalised
 * cloud-in-cell reconstruction of Eq. (reconstruction); velocity moments give
 * the charge density; the sinc-softened spectral Poisson solve of
 * Eq. (poissonk)/(kappasoftening) gives E; E goes back to the markers with the
 * same area weighting.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is DEVICE memory owned by the caller unless its name
 *    ends in _host.  libavl never allocates or frees device memory; all of its
 *    device state lives in the caller's workspace (avl_reconstruct_noalloc
 *    alone uses a static device array of the library instead).  The handle
 *    itself is a small host object owned by libavl and released by avl_destroy.
 *  - Work is enqueued on the handle's HIP stream (hipStream_t passed as void*,
 *    NULL = legacy default stream) and is asynchronous unless stated; results
 *    are valid after the stream is synchronised.  Calls on one handle are not
 *    thread-safe; distinct handles are independent.
 *  - Grid layout (Sec. 3.1, Fig. "phasespace"): x in [0, L) periodic with nx
 *    cells (dx = L/nx); velocity component d has nv[d] cells on
 *    [vmin[d], vmax[d]); all grid values sit at cell centres.  Phase-space
 *    arrays are velocity-major, index ((jz*nv[1] + jy)*nv[0] + jx)*nx + i
 *    (1D-1V: j*nx + i).  Spatial arrays (rho, E) have nx entries.
 *  - Marker arrays are structure-of-arrays FP64: x[n], v[vdim*n] (component d
 *    of marker l at v[d*n + l]), f[n] (the phase-space density each marker
 *    carries, its "weight" in the paper's words, Sec. 2).
 *  - Units are the caller's: acceleration is (q/m) E, Poisson's equation is
 *    dE/dx = c_p * rho (c_p = 4*pi in the paper's CGS units, Eq. (poisson)).
 *  - Return values: AVL_OK (0) or a negative avl_rc.  Host-side validation
 *    runs before anything is enqueued, so an error return leaves the handle and
 *    the device untouched, except AVL_EDEVICE (a HIP call failed).
 */
#ifndef AVL_H_
#define AVL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef enum {
    AVL_OK = 0,
    AVL_EINVAL = -1,      /* bad argument or configuration value */
    AVL_ESIZE = -2,       /* workspace too small, or a size over the supported range */
    AVL_EALIGN = -3,      /* workspace not 256-byte aligned, or an array not 8-byte aligned */
    AVL_ESTATE = -4,      /* call not valid in the handle's current state */
    AVL_EDEVICE = -5,     /* a HIP runtime call failed */
    AVL_ENOTSUP = -6,     /* configuration outside what this build implements */
    AVL_ENONFINITE = -7,  /* device kernels saw a non-finite marker or field value */
    AVL_EINTERNAL = -8    /* device consistency check failed (sort slots, encoding range) */
} avl_rc;

/* Marker storage form.
 *  AVL_FP64: plain form, markers and grid in FP64.
 *  AVL_FP32: each marker stores the integer index of the cell whose centre is
 *            its lower-left cloud neighbour plus FP32 offsets in [0,1) from that
 *            centre (a along x, b along each velocity component) and an FP32 f;
 *            the push works in cell units, the f grid is FP32; rho and the field
 *            solve stay FP64.  In 1D-3V the vy and vz clouds of every marker
 *            must touch the velocity grid (they never move; a marker outside
 *            raises AVL_EINTERNAL at the next avl_check), and the x-velocity
 *            index may leave the grid by at most 32 rows; in 1D-1V the
 *            velocity index may leave it by up to 2^(30 - log2 nx) - 2 rows.
 *            Markers beyond these ranges are clamped into them and flagged
 *            (AVL_EINTERNAL at the next avl_check). */
typedef enum { AVL_FP64 = 0, AVL_FP32 = 1 } avl_precision;

/* Options.  The reconstruction sums, per run of markers sharing a cell, the
 * moments S_f, S_af, S_bf, S_abf, S_a, S_b, S_ab of the offsets (from which
 * the four cloud-in-cell corner sums follow exactly); by default these
 * accumulate in FP64 in both forms, each term rounded down onto a grid fitted
 * to the run, so that the sums do not depend on the order of the run's markers
 * and every result is reproducible bit for bit.
 *  AVL_OPT_KAHAN32: FP32 form of 1D-1V only: accumulate the four corner sums
 *                   of N and D directly in FP32 with compensated (Kahan)
 *                   summation instead (reproducible to rounding, not bit for
 *                   bit: the order of a run's markers varies from run to run;
 *                   AVL_ENOTSUP for 1D-3V, whose reconstruction always sums in
 *                   FP64). */
typedef enum { AVL_OPT_KAHAN32 = 1 } avl_option;

typedef struct avl_config {
    int32_t vdim;        /* 1 (1D-1V) or 3 (1D-3V) */
    int32_t nx;          /* power of two in [8, 4096] */
    int32_t nv[3];       /* velocity cells per component, each >= 2 (only [0, vdim) used) */
    int32_t precision;   /* avl_precision */
    int32_t first_kick;  /* 0: first velocity update is a full dt from v^0; 1: half dt */
    int32_t options;     /* bit set of avl_option, 0 for the defaults */
    int64_t n_markers;   /* number of markers n, 0 <= n < 2^31 */
    double L;            /* domain length, finite > 0 */
    double vmin[3];      /* lower velocity bound per component */
    double vmax[3];      /* upper velocity bound, > vmin */
    double dt;           /* time step, finite > 0 */
    double q;            /* species charge (enters rho) */
    double m;            /* species mass (acceleration is q/m * E), finite != 0 */
    double c_p;          /* Poisson constant, finite > 0 */
    int32_t tune[4];     /* kernel tuning knobs, 0 = library default (results do not depend on
                            them beyond summation order):
                            [0] target velocity rows per 1D-1V reconstruction task, 1..256;
                            [1] row form of the FP32 1D-1V reconstruction: 1 dense rows (every
                                register load issued), 2 sparse rows (loads past a row segment
                                skipped); the default takes sparse rows when a segment averages
                                below 0.6 of the register capacity; ignored by other forms;
                            [2] resident blocks per compute unit of the FP32 1D-1V tiled count
                                and scatter passes, 1..64 (at most what fits; the default is
                                what fits);
                            [3] reserved, must be 0 */
    double B[3];         /* uniform background magnetic field (1D-3V, AVL_FP64 only; all zero
                            otherwise): the acceleration is (q/m)(E + v x B), E along x, and
                            the push is the Boris scheme (Sec. 2, magnetised 1D-3V: a half
                            electric kick, a rotation about B, a half electric kick).  The
                            gyration must take at least 2 pi steps, |q/m| |B| dt <= 1
                            (AVL_EINVAL otherwise); AVL_ENOTSUP with AVL_FP32 */
} avl_config;

typedef struct avl_handle avl_handle;

/* Bytes of device workspace a handle for `cfg` needs (0 if cfg is invalid).
 * Holds two marker buffers (the sort is out of place), per-cell counts and
 * offsets, the f grid, partial and final rho, E, the field-solve tables and a
 * diagnostics ring. */
size_t avl_workspace_bytes(const avl_config* cfg);

/* Create a handle and load the markers (Sec. 2 marker loading; Sec. 3.1: the
 * field starts from the loaded state).  Copies x, v, f (FP64, n markers, SoA as
 * above; x must lie in [0, L)) into `workspace` (>= avl_workspace_bytes,
 * 256-byte aligned, caller-owned for the handle's lifetime), converting to the
 * FP32 form if asked, sorts them by cell, then computes f^0, rho^0 and E^0 so
 * that the first avl_step pushes with E^0.  `stream` is a hipStream_t.
 * Synchronises the stream once to check the loaded markers: returns
 * AVL_EINVAL if an x lies outside [0, L) or any value is non-finite. */
int avl_init(const avl_config* cfg, void* workspace, size_t ws_bytes, void* stream,
             const double* x, const double* v, const double* f, avl_handle** out);

/* Gather and push (Sec. 2, the final paragraph of the method overview): each
 * marker gets E at its position by the same area weighting as the
 * reconstruction, then v += (q/m) E dt (x velocity only) and x += v dt, wrapped
 * into [0, L).  Uses E (nx values) if non-NULL, else the handle's current
 * field.  Marker order is preserved; the handle's f, rho and E become stale.
 * The first push after avl_init uses a half kick when cfg.first_kick = 1. */
int avl_push(avl_handle* h, const double* E);

/* Reorder the markers by cell (a counting sort keyed on the cell whose centre
 * is each marker's lower-left cloud neighbour).  Needed before a
 * reconstruction; avl_reconstruct calls it itself when the order is stale. */
int avl_sort(avl_handle* h);

/* Weight-normalised reconstruction, Eq. (reconstruction): for every phase
 * cell g, N_g = sum_l alpha_gl f_l, D_g = sum_l alpha_gl, f_g = N_g / D_g with
 * cloud-in-cell area weights alpha (Sec. 2, Fig. "interpolation"); x periodic,
 * cloud parts outside the velocity range dropped; f_g = 0 where D_g = 0.
 * 1D-1V uses area weights in (x, vx); 1D-3V the volume weights of a cloud of
 * one cell in (x, vx, vy, vz), 16 cells per marker.
 * f_out and D_out (may be NULL) receive G = nx*prod(nv) values in the storage
 * precision (double for AVL_FP64, float for AVL_FP32). */
int avl_reconstruct(avl_handle* h, void* f_out, void* D_out);

/* Charge-density moment (Sec. 2 overview; Sec. 3.4 spatial output):
 * rho_i = q * prod(dv) * sum over velocity cells of f at x cell i, FP64, from
 * the last reconstruction.  rho_out (may be NULL) receives nx doubles.
 * AVL_ESTATE if f is stale (markers pushed since the last reconstruction). */
int avl_moments(avl_handle* h, double* rho_out);

/* Spectral field solve, Eq. (poissonk) with Eq. (kappasoftening): E_hat_m =
 * -i c_p kappa_m / K_m^2 rho_hat_m, kappa = k sinc(k dx), K^2 = k^2
 * sinc^2(k dx/2), E_hat_0 = 0 (DC removal) and the Nyquist mode zeroed.  Takes
 * rho (nx doubles) or, if NULL, the handle's rho from avl_moments.  The result
 * becomes the handle's field; E_out (nx doubles) and W_out (1 double: the field
 * energy sum E_i^2 dx / (2 c_p), Sec. 3.4) may be NULL.  FP64 throughout. */
int avl_poisson(avl_handle* h, const double* rho, double* E_out, double* W_out);

/* `nsteps` full steps: gather+push with E^n, sort, reconstruct f^{n+1},
 * rho^{n+1}, solve E^{n+1}.  diag_out (may be NULL) receives 2*nsteps doubles,
 * per step the field energy W and the amplitude (2/nx)|sum_i E_i e^{-2 pi i
 * i/nx}| of the longest-wavelength mode of E (Sec. 4.2).  AVL_ESTATE unless
 * the handle holds a current field (after avl_init, avl_poisson or a step). */
int avl_step(avl_handle* h, int32_t nsteps, double* diag_out);

/* Same as avl_step, replaying a HIP graph of one step captured on first use
 * (a fixed launch sequence; identical results to avl_step). */
int avl_step_graph(avl_handle* h, int32_t nsteps, double* diag_out);

/* Export the markers in FP64 (SoA as in avl_init) in the current storage
 * order.  The FP32 form is converted: x = (i + 1/2 + a) dx, v = vmin + (j +
 * 1/2 + b) dv with (i, j) the stored cell. */
int avl_get_markers(avl_handle* h, double* x, double* v, double* f);

/* Replace the markers (FP64 SoA, same count, x in [0, L)), e.g. to resume
 * from a checkpoint taken with avl_get_markers: they are re-sorted and f, rho
 * and E recomputed as in avl_init, while the step count and the first-kick
 * state carry on.  Synchronises. */
int avl_set_markers(avl_handle* h, const double* x, const double* v, const double* f);

/* Copy the handle's current field (nx doubles) and charge density. */
int avl_get_field(avl_handle* h, double* E_out, double* rho_out);

/* Thermodynamic and field diagnostics of the current state (the quantities
 * the paper writes per output step, Sec. 3.4 "Thermodynamical quantities" and
 * "Spatial output"), from the last reconstruction f, its charge density rho
 * and the field E solved from it (AVL_ESTATE otherwise, e.g. after a push
 * without a new reconstruction and solve).  Cell-centre velocities v_g,
 * dV = dx * prod(dv):
 *   out[0] Ee    = sum_i E_i^2 dx / (2 c_p)            (field energy)
 *   out[1] Ekin  = m/2 * sum_g f_g |v_g|^2 dV          (kinetic energy)
 *   out[2] Etot  = Ee + Ekin
 *   out[3] N     = sum_g f_g dV                        (integral of f)
 *   out[4] S     = sum_{g: f_g > 0} f_g log(f_g) dV    (entropy integral as the paper defines it)
 *   out[5] P     = m * sum_g f_g v_x,g dV              (momentum)
 * j_out (nx doubles, may be NULL): current density j_i = q prod(dv) sum_j v_x f_ij.
 * drho_out (nx doubles, may be NULL): the field solver's residual charge
 * (rho_i - mean(rho)) - (E_{i+1} - E_{i-1}) / (2 dx c_p) (the mean is the
 * neutralising background; centred difference, periodic).
 * out: 6 doubles of device memory.  Sums are FP64 in a fixed order. */
int avl_diagnostics(avl_handle* h, double* out, double* j_out, double* drho_out);

/* ---- Several species in one self-consistent field (Sec. 2: rho is the sum
 * over species of q_s prod(dv_s) sum_j f_s; every species is pushed by the one
 * field; e.g. electrons and mobile ions) ---- */
typedef struct avl_multi avl_multi;

/* Device workspace bytes of a group of nspecies species on an x grid of nx
 * cells (0 if out of range: 1..64 species). */
size_t avl_multi_workspace_bytes(int32_t nspecies, int32_t nx);

/* Group n existing handles (each with its own charge, mass, velocity grid,
 * storage form and markers) that share nx, L, c_p, dt, first_kick and the
 * stream (AVL_EINVAL otherwise).  The handles stay owned by the caller and
 * must outlive the group; the field of every handle is replaced by the field
 * of the total charge density (the neutralising background is the removed
 * mean, as for one species).  AVL_ESTATE if a handle has no current rho. */
int avl_multi_init(avl_handle* const* hs, int32_t n, void* workspace, size_t bytes, avl_multi** out);

/* nsteps steps of every species in the shared field: push and sort each, then
 * reconstruct each, sum the charge densities in species order, solve once and
 * give every species the field.  diag_out (2*nsteps doubles or NULL) receives
 * the field energy and mode-1 amplitude per step, as avl_step does.  Each
 * handle's rho is its own species' charge density; avl_diagnostics on a handle
 * reports that species' kinetic quantities with the total field's energy. */
int avl_multi_step(avl_multi* m, int32_t nsteps, double* diag_out);

/* Release the group (not its handles). */
int avl_multi_destroy(avl_multi* m);

/* Number of full steps taken since the markers were loaded. */
int64_t avl_step_count(const avl_handle* h);

/* Synchronise the stream and report sticky device-side conditions:
 * AVL_ENONFINITE, AVL_EINTERNAL or AVL_OK. */
int avl_check(avl_handle* h);

/* The same query under its other name: identical behaviour and result. */
int avl_status(avl_handle* h);

/* Rebind the handle to another stream (hipStream_t). */
int avl_set_stream(avl_handle* h, void* stream);

/* Kernel timing with HIP events recorded on the handle's stream around every
 * launch of the named kernel class while enabled (see AVL_K_* below).
 * avl_kernel_time synchronises and returns the summed milliseconds and the
 * number of launches since timing was enabled. */
enum { AVL_K_PUSH_COUNT = 0, AVL_K_SCAN = 1, AVL_K_SCATTER = 2, AVL_K_RECONSTRUCT = 3,
       AVL_K_FIELD = 4 /* rho from the reconstruction's partials + field solve */, AVL_K_STEP = 5,
       AVL_K_COUNT = 6 };
int avl_timing(avl_handle* h, int enable);
int avl_kernel_time(avl_handle* h, int kernel, double* ms_total, int64_t* launches);

/* Algorithmic bytes one launch of the named kernel class moves for this
 * handle's configuration (what the kernel must read and write, excluding
 * re-reads): used to express achieved bandwidth.  For AVL_K_STEP it is the
 * method's own traffic of one step with the sort left out (the push reads and
 * writes positions and velocities; the reconstruction reads every marker's
 * offsets and f and the run offsets and writes the f grid); the sort's bytes
 * are the sum of the AVL_K_PUSH_COUNT, AVL_K_SCAN and AVL_K_SCATTER entries. */
double avl_kernel_bytes(const avl_handle* h, int kernel);

/* Measurement aid: copy `bytes` (multiple of 16) from src to dst with a plain
 * streaming kernel on `stream`; calibrates achievable HBM bandwidth and the
 * hardware byte counters. */
int avl_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/* Text for a status code. */
const char* avl_strerror(int status);

/* Release the handle (host memory only; the workspace stays the caller's). */
int avl_destroy(avl_handle* h);

/* ---------------------------------------------------------------------------
 * Batches: many independent 1D-1V instances (a parameter scan) stepped
 * together.  Each step of the batch is six launches that cover every
 * instance (count, scan, scatter, reconstruction, rho, field solve), replayed
 * as a HIP graph; each launch holds a work list of (instance, block or task)
 * items, so uneven instances share the GPU without one launch per instance.
 * The method per instance is exactly the single-handle step above.
 * ------------------------------------------------------------------------- */
typedef struct avl_batch avl_batch;

/* Device workspace for `count` instances (1 <= count <= 4096) with
 * configurations cfgs[0..count) (0 if any is invalid, not 1D-1V, or if they
 * differ in precision, options or first_kick). */
size_t avl_batch_workspace_bytes(const avl_config* cfgs, int32_t count);

/* Create a batch.  Instance i is initialised as by avl_init with cfgs[i] and
 * the markers that follow instance i-1's in the concatenated device arrays x,
 * v, f (FP64; instance i's markers are elements [o_i, o_i + n_i) with
 * o_i = n_0 + ... + n_{i-1}, n_i = cfgs[i].n_markers).  `workspace` as for
 * avl_init (256-byte aligned, >= avl_batch_workspace_bytes, caller-owned).
 * Errors as avl_init; AVL_ENOTSUP for combinations the batch does not take. */
int avl_batch_init(const avl_config* cfgs, int32_t count, void* workspace, size_t ws_bytes, void* stream,
                   const double* x, const double* v, const double* f, avl_batch** out);

/* `nsteps` steps of every instance.  diag_out (NULL or count*nsteps*2
 * doubles, instance-major) receives each instance's per-step W and mode-1
 * amplitude as avl_step does. */
int avl_batch_step(avl_batch* b, int32_t nsteps, double* diag_out);

/* Instance i as a handle for the per-handle calls (avl_get_field,
 * avl_get_markers, avl_reconstruct, avl_check, ...), owned by the batch:
 * do not destroy it.  NULL if i is out of range. */
avl_handle* avl_batch_instance(avl_batch* b, int32_t i);

/* Number of instances (-1 for NULL). */
int avl_batch_count(const avl_batch* b);

/* avl_check over every instance (the first failure is returned). */
int avl_batch_check(avl_batch* b);

/* Release the batch and its instance handles. */
int avl_batch_destroy(avl_batch* b);

/* ---------------------------------------------------------------------------
 * Adjoint (1D-1V, either storage form): the gradient of the time-integrated field
 * energy J = sum_{n=1..nsteps} sum_i (E_i^n)^2 dx dt with respect to the
 * marker weights f_l, by the reverse of every stage of the step (gather,
 * push, reconstruction f = N/D, moments, spectral solve; Sec. 2 and
 * Eq. (reconstruction), Eq. (poissonk)).  Parameters of the initial
 * distribution enter through f_l = f0(x_l, v_l), so dJ/dtheta =
 * sum_l dJ/df_l df_l/dtheta.
 * ------------------------------------------------------------------------- */

/* Device recording workspace for an adjoint run of `nsteps` steps that keeps
 * a checkpoint every `every` steps: the checkpoints (the raw marker buffer),
 * one segment's states (FP64 coordinates) and grids, and the adjoint arrays
 * (0 if the configuration is not 1D-1V or nsteps, every < 1).  The reverse
 * sweep works on FP64 coordinates; for the FP32 form they are the exact
 * conversions of the stored cell and offsets. */
size_t avl_adjoint_workspace_bytes(const avl_config* cfg, int32_t nsteps, int32_t every);

/* Load (x, v, f) into h as avl_set_markers does but from step 0, run nsteps
 * steps keeping a checkpoint every `every` steps in `rec` (device, 256-byte
 * aligned, >= avl_adjoint_workspace_bytes, caller-owned), then sweep back
 * segment by segment, recomputing each from its checkpoint.  Writes J to
 * J_out (1 device double) and dJ/df_l for every marker, in the order of f, to
 * grad_f (n device doubles).  Synchronises.  Afterwards h holds a recomputed
 * state inside the first segment (reload before further stepping).
 * AVL_ENOTSUP for 1D-3V; AVL_ESTATE while kernel timing is enabled. */
int avl_adjoint(avl_handle* h, const double* x, const double* v, const double* f, int32_t nsteps, int32_t every,
                void* rec, size_t rec_bytes, double* J_out, double* grad_f);

/* The reverse stages of one step, one call each, on caller-supplied states
 * (avl_adjoint chains the same kernels).  Each is the transpose of the
 * linearised forward stage, so <J du, lam> = <du, J^T lam> holds for any du,
 * lam.  All arrays are device memory, caller-owned, 8-byte aligned; outputs
 * are overwritten; enqueued on the handle's stream.  AVL_ESTATE while kernel
 * timing is enabled.  The field adjoint of the push is summed as integers on a
 * grid set by its largest term (see the header of the reverse kernels), so
 * results do not depend on marker order.
 *
 * Reconstruction f = N/D (Eq. (reconstruction)) and moments
 * rho_i = q prod(dv) sum_j f_ij (Sec. 2), reversed: rho_bar (nx) gives
 * f_bar = dJ/df_l and, when lam_x and lam_v are both non-NULL, the position
 * and velocity adjoints dJ/dx_l, dJ/dv_l (n each, in the order of x, v, f).
 * x, v, f: the state's markers (FP64, n = cfg n_markers, any order); f_grid,
 * D_grid: that state's f and D grids in the storage precision, as
 * avl_reconstruct writes them for these markers.  Cells with D = 0 carry
 * nothing.  1D-1V only (AVL_ENOTSUP otherwise). */
int avl_adjoint_deposit(avl_handle* h, const double* x, const double* v, const double* f, const void* f_grid,
                        const void* D_grid, const double* rho_bar, double* f_bar, double* lam_x, double* lam_v);

/* Gather + kick + drift (Sec. 2: E interpolated to the marker with the
 * cloud-in-cell weights, v' = v + (q/m) E dt kick, x' = x + v' dt), reversed:
 * from the adjoints lam_x_in, lam_v_in of (x', v') and the field E (nx) the
 * push used, the adjoints lam_x, lam_v of (x, v) and E_bar = dJ/dE (nx).  x:
 * positions before the push (FP64, n); kick: the fraction of dt of the
 * velocity update (1, or 1/2 for a half first kick).  lam_x may equal
 * lam_x_in and lam_v may equal lam_v_in (in place).  1D-1V only. */
int avl_adjoint_push(avl_handle* h, const double* x, const double* E, double kick, const double* lam_x_in,
                     const double* lam_v_in, double* lam_x, double* lam_v, double* E_bar);

/* The spectral solve E = P rho (Eq. (poissonk), softened by
 * Eq. (kappasoftening), mean of rho removed), reversed: rho_bar = P^T mu =
 * -P mu (P is a real convolution whose transfer function is odd and
 * imaginary).  mu and rho_bar: nx doubles each, distinct arrays. */
int avl_adjoint_field(avl_handle* h, const double* mu, double* rho_bar);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * reconstruction of avl_reconstruct for a marker set given directly (loaded
 * and sorted as avl_init does it), with no handle and no workspace.
 * ------------------------------------------------------------------------- */

/* Size of the library's static scratch array per GPU (64 MiB): it holds the
 * two marker buffers, the per-cell counts and offsets, the sort's tile totals
 * and the reconstruction's charge partials of one call. */
#define AVL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* Markers x, v, f (FP64, SoA as for avl_init; x in [0, L), all finite) are
 * converted to cfg's storage form, sorted by cell and reconstructed:
 * f_out (required) and D_out (may be NULL) receive G = nx*prod(nv) values in
 * the storage precision (double for AVL_FP64, float for AVL_FP32), equal bit
 * for bit to what avl_init followed by avl_reconstruct gives for the same
 * markers and configuration.  Every step is a kernel launched on `stream`
 * (a hipStream_t); the call allocates nothing (no hipMalloc, no host
 * allocation), copies nothing from the host and does not synchronise, so it
 * may be captured into a HIP graph.  The inputs are not validated on the
 * device (avl_init's checks need a synchronisation): values outside the rules
 * above give meaningless output, never out-of-bounds accesses.
 * All scratch lives in one static device array per GPU, kept until the
 * process ends: every call on a GPU shares it, so calls that overlap on one
 * GPU (two streams, two host threads, or a graph replayed while another call
 * runs) race and must be serialised by the caller.  The first call on each
 * device looks up the array's device address (not a stream operation).
 * Errors: avl_init's configuration errors; AVL_EINVAL for a NULL f_out or a
 * missing marker array; AVL_EALIGN for arrays not 8-byte aligned; AVL_ESIZE
 * when the configuration needs more than AVL_NOALLOC_SCRATCH_BYTES (about
 * 1.3 million FP64 1D-1V markers); AVL_EDEVICE if a launch or the lookup
 * fails. */
int avl_reconstruct_noalloc(const avl_config* cfg, void* stream, const double* x, const double* v,
                            const double* f, void* f_out, void* D_out);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif
#endif /* AVL_H_ */
