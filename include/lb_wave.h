/*
 * lb_wave.h -- C ABI of the MI355X wave lattice Boltzmann library that
 * computes the time-averaged acoustic radiation force on density-matched
 * compressible objects.
 *
 * Method: Castro-Avila, Malgaretti, Harting, Munoz, "A lattice Boltzmann
 * approach for acoustic manipulation" (arXiv 2404.02346).
 *   - lattice, equilibrium, collision (tau = 1/2), advection:
 *       Sec. "Lattice-Boltzmann for acoustics", eqs. MacroscopicFields,
 *       LBM-Collision, LBM-Advection, feq_waves (D2Q5 with c_s^2 = 1/3,
 *       D3Q7 with c_s^2 = 1/4);
 *   - source sheet and damped walls: eqs. imposingfields, bounce-back, and
 *       the set-up of Sec. "Results and discussion" (absorbing wall x = 0,
 *       source x = 1, reflector x = Lx-1, periodic y and z);
 *   - object: per-cell sound speed of eq. sound_speed_object, read with
 *       c = c_p inside and c = c0 outside;
 *   - measurement: kernel interpolation (eq. InterpolatedFields, 3-point
 *       kernel applied as a tensor product) onto surface elements, surface
 *       integral eq. arf_integral_LBM at every step, time average over the
 *       steps t >= avg_start.
 *
 * Conventions
 *   - All functions have C linkage and return an lb_status (0 = success,
 *     negative = error) unless stated otherwise; lb_last_error() gives a
 *     thread-local message for the last failure.
 *   - Pointers are HOST pointers unless the name starts with dev_.
 *   - Lattice units: dx = dt = 1.  Node (x, y, z) sits at integer
 *     coordinates 0 <= x < nx etc.; cell index (z*ny + y)*nx + x.
 *   - Velocity order 0, +x, -x, +y, -y, +z, -z (Q = 5 in 2D, 7 in 3D).
 *   - A "state" is f^new, the post-collision populations before advection,
 *     which is the instant the paper reads results at.  Step t advects the
 *     state of step t-1, collides, applies the sheets and measures F(t)
 *     from rho1, J1 of the advected populations.
 *   - The library never allocates device memory: the caller passes one
 *     device workspace (e.g. a torch uint8 tensor) of at least
 *     lb_wave_workspace_bytes() bytes, 256-byte aligned, which it owns and
 *     must keep alive until lb_wave_destroy().  Work is enqueued on the
 *     caller's HIP stream.
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef LB_WAVE_H
#define LB_WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage precision of the populations.  F64 and F32 compute in their own
 * precision; F16 and BF16 store 16-bit values (times a power-of-two scale)
 * and compute the collision in FP32.  Interpolation and the surface integral
 * are FP64 in every mode; the time accumulator is FP64. */
typedef enum { LB_F64 = 0, LB_F32 = 1, LB_F16 = 2, LB_BF16 = 3 } lb_storage;

/* Boundary along x: the paper's driven sheets, or periodic (no sheets). */
typedef enum { LB_XBC_DRIVEN = 0, LB_XBC_PERIODIC = 1 } lb_xbc;

/* Where the wave comes from.  LB_SRC_SHEET: the driven sheet x = 1 (none in
 * periodic mode).  LB_SRC_POINT: one node, the oscillating point source of
 * the paper's first validation (Sec. "Lattice-Boltzmann for acoustics",
 * eq. waves_with_pointSource): after every collision the node src_cell
 * takes f^eq(rho_a sin(omega t), J1) with J1 its own pre-collision momentum,
 * the rule of the source sheet (eq. imposingfields).  A point source needs
 * periodic x (no sheets) and keeps one lattice step per launch. */
typedef enum { LB_SRC_SHEET = 0, LB_SRC_POINT = 1 } lb_source;

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,      /* bad argument, shape or parameter */
    LB_ENOMEM = -2,      /* workspace too small or misaligned */
    LB_EUNSTABLE = -3,   /* some c(x) > 1/sqrt(dim): the tau = 1/2 scheme grows */
    LB_EGEOMETRY = -4,   /* a surface stencil touches an x sheet or leaves the box */
    LB_EDEVICE = -5,     /* a HIP call failed */
    LB_ENAN = -6,        /* a measured force was not finite */
    LB_EEMPTY = -7       /* no step has been accumulated yet */
} lb_status;

/* One problem instance (one box with one object). */
typedef struct lb_wave_desc {
    int32_t dim;                /* 2 (D2Q5) or 3 (D3Q7) */
    int32_t nx, ny, nz;         /* lattice size; nz = 1 when dim = 2 */
    int32_t storage;            /* lb_storage; identical for all instances of a handle */
    int32_t xbc;                /* lb_xbc */
    double c0, rho0;            /* fluid sound speed (cells/step) and mean density */
    const double *c_field;      /* optional nx*ny*nz per-cell sound speed (cell index
                                   order); NULL selects the analytic object below */
    double obj_center[3];       /* object centre r0 (z ignored in 2D) */
    double obj_radius;          /* R_p */
    double obj_cp;              /* sound speed inside the object c_p */
    double obj_d;               /* "square thickness" d of the tanh profile (paper: 4) */
    double rho_a;               /* source amplitude: rho1 = rho_a sin(omega t) on the source */
    double omega;               /* drive angular frequency (rad/step) */
    double wall_phi;            /* bounce-back damping Phi in [0, 1) (paper: 0.99) */
    int32_t n_surf;             /* number of surface elements N (may be 0) */
    const double *surf_xyz;     /* N*3 element centres R_k */
    const double *surf_normal;  /* N*3 outward unit normals n_k */
    const double *surf_area;    /* N element sizes dS_k (length in 2D, area in 3D) */
    int64_t avg_start;          /* F(t) enters the average for t >= avg_start */
    int64_t max_steps;          /* the instance freezes after this many steps; <= 0: never */
    int64_t trace_steps;        /* keep F(t) for t < trace_steps (0: no trace) */
    int32_t src_kind;           /* lb_source (0, the sheet, for descriptors set to zero) */
    int32_t src_cell[3];        /* LB_SRC_POINT: the source node (x, y, z); z = 0 in 2D */
} lb_wave_desc;

typedef struct lb_wave lb_wave;  /* opaque handle */

/* Check descriptors on the host only (no device call).  Returns LB_OK or the
 * first error: LB_EINVAL (shapes, dim, storage mismatch between instances,
 * missing surface arrays, rho0 <= 0, wall_phi outside [0, 1), nx < 3 with
 * driven x, a point source with driven x or a source node outside the
 * lattice), LB_EUNSTABLE (c0, c_p or any c_field value above 1/sqrt(dim),
 * the stability bound of the tau = 1/2 scheme), LB_EGEOMETRY (a 3-point
 * stencil reaches x < 2 or x > nx-2 in driven mode, where the sheets change
 * the moments, or leaves 0 <= x < nx in periodic mode). */
int lb_wave_check(const lb_wave_desc *descs, int32_t n_inst);

/* Device bytes needed for n_inst instances (0 if lb_wave_check fails). */
size_t lb_wave_workspace_bytes(const lb_wave_desc *descs, int32_t n_inst);

/* Create a handle: validates, copies every host array (the caller may free
 * them on return), lays out the workspace, builds the compact c^2 tables
 * and surface stencils, and zeroes the state (f^new of step -1 = 0) and the
 * accumulators, all on `hip_stream` (hipStream_t, NULL = default stream).
 * The sound speed of an analytic object is eq. sound_speed_object of Sec.
 * "Wave-particle interaction and interpolation" (c_p inside, c0 outside: the
 * printed sign is inverted, see the descriptor); each surface element's
 * stencil is the 3 x 3 (x 3) nodes of the 3-point kernel of eq.
 * InterpolatedFields, taken as a tensor product of the printed 1D kernel,
 * with its weights precomputed.
 * dev_workspace must be 256-byte aligned device memory of workspace_bytes
 * >= lb_wave_workspace_bytes().  On success *out receives the handle. */
int lb_wave_create(const lb_wave_desc *descs, int32_t n_inst, void *dev_workspace,
                   size_t workspace_bytes, void *hip_stream, lb_wave **out);

/* Enqueue n_steps steps for every instance (an instance past max_steps is
 * left untouched).  A step is the scheme of Sec. "Lattice-Boltzmann for
 * acoustics": moments (eq. MacroscopicFields), BGK collision with tau = 1/2
 * towards the wave equilibrium with the local c (eqs. LBM-Collision and
 * feq_waves), the damped bounce-back walls at x = 0 and nx-1 (eq.
 * bounce-back) and the imposed density rho_a sin(omega t) at x = 1 (eq.
 * imposingfields) in driven mode, then advection (eq. LBM-Advection); the
 * force F(t) of each step is measured as lb_surface_force describes.
 * Asynchronous: returns after enqueueing.  Returns LB_ENAN if a previous
 * lb_surface_force() found a non-finite force. */
int lb_wave_step_n(lb_wave *h, int64_t n_steps);

/* Synchronise the stream and return, per instance in the order given to
 * create, the time average of F(t) over the accumulated steps
 * (F_avg: n_inst*3 doubles, required) and the number of accumulated steps
 * (n_accum: n_inst, may be NULL).  F(t) is the surface integral of eq.
 * arf_integral_LBM over the surface elements, with rho1 and J1 interpolated
 * to each element (eq. InterpolatedFields) from the step's fields; the
 * average over the steps t >= avg_start follows Sec. "Results and
 * discussion" (the force is evaluated every step and averaged once the wave
 * has settled).  LB_EEMPTY if some instance has none (its F_avg is then 0),
 * LB_ENAN if some force was not finite. */
int lb_surface_force(lb_wave *h, double *F_avg, int64_t *n_accum);

/* Release the handle (NULL-safe).  Does not free the caller's workspace. */
int lb_wave_destroy(lb_wave *h);

/* Thread-local message of the last failure ("" if none). */
const char *lb_last_error(void);

/* ---- inspection and control (tests, benchmarks) ---- */

/* Steps enqueued so far (global step counter t). */
int lb_wave_steps_done(const lb_wave *h, int64_t *t);

/* Zero the state, the step counter and the accumulators (stream-ordered). */
int lb_wave_reset(lb_wave *h);

/* Copy the current state of instance `inst` to/from the host as FP64
 * cells x Q (array-of-structures, cell index order, unscaled).  Both
 * synchronise the stream.  set_state replaces the state the next step
 * advects (f^new of the previous step); 16-bit storage rounds it. */
int lb_wave_get_state(lb_wave *h, int32_t inst, double *host_fnew);
int lb_wave_set_state(lb_wave *h, int32_t inst, const double *host_fnew);

/* Copy F(t) for t = 0 .. n-1 (n <= trace_steps) of instance `inst` to
 * host (n*3 doubles); synchronises the stream. */

/* rho1 = sum_i f_i (eq. MacroscopicFields) of instance `inst` at n_cells
 * cells of its current state (f^new of the last step, whose moments equal
 * the pre-collision ones off the x sheets), FP64, unscaled.  dev_cells:
 * n_cells int64 cell indices (z ny + y) nx + x in device memory; dev_out:
 * n_cells doubles in device memory; an index outside the lattice gives NaN.
 * Asynchronous on the handle's stream (read after the steps enqueued before
 * it).  LB_EINVAL for a bad instance, n_cells < 0 or a NULL pointer. */
int lb_wave_probe_rho(lb_wave *h, int32_t inst, const int64_t *dev_cells, int32_t n_cells,
                      double *dev_out);
int lb_wave_force_trace(lb_wave *h, int32_t inst, double *host_F, int64_t n);

/* Where the populations live inside the workspace (for zero-copy reads):
 * offset in bytes of population plane 0 of the current state buffer,
 * bytes between planes, elements per row (pitch >= nx) and the storage
 * scale s (stored value = s * f). */
typedef struct lb_state_view {
    size_t offset_bytes;
    size_t plane_bytes;
    int32_t pitch;
    int32_t elem_bytes;
    double scale;
} lb_state_view;
int lb_wave_state_view(const lb_wave *h, int32_t inst, lb_state_view *v);

/* Variant of the step kernel:
 *   cells_per_lane 1, 2 or 4: contiguous cells a lane moves with one vector
 *     load/store per population (a wavefront covers 64 * cells_per_lane cells);
 *   x_mode 0: the +x/-x neighbours are shifted across lanes; 1: they are read
 *     with a vector load offset by one element (4- and 8-byte storage only);
 *   nontemporal 0: plain loads and stores, 1: non-temporal stores,
 *     2: non-temporal loads and stores.
 * Every variant computes bit-identical results.  lb_wave_autotune times every
 * valid variant, and two steps per launch where allowed, for n_trial steps
 * (rounded up to even) on the handle's own instances, keeps the fastest,
 * then resets the state (lb_wave_reset); best_ms (may be NULL) receives the
 * winning time per step in ms.  set_tile/get_tile change or read
 * cells_per_lane only. */
int lb_wave_set_variant(lb_wave *h, int32_t cells_per_lane, int32_t x_mode, int32_t nontemporal);
int lb_wave_get_variant(const lb_wave *h, int32_t *cells_per_lane, int32_t *x_mode,
                        int32_t *nontemporal);
int lb_wave_set_tile(lb_wave *h, int32_t cells_per_lane);
int lb_wave_get_tile(const lb_wave *h, int32_t *cells_per_lane);
int lb_wave_autotune(lb_wave *h, int32_t n_trial, double *best_ms);

/* Lattice steps per launch: 1 (step_kernel, the default) or 2 (a fused
 * kernel that advances t -> t + 2 with step t's values held on chip, reading
 * and writing the state about once per two steps).  Two steps per launch
 * need every instance 3D with driven x sheets and ny a multiple of the row
 * block, R * 4 / nw rows (R = 4 rows per row group for FP32 and 2 for the
 * other storage types; nw = pitch / 64 wavefronts cover a row up to 256
 * cells; longer rows run in strips of 254 cells, nw = 4); otherwise
 * LB_EINVAL.  Results are bit-identical either way; steps where an instance stops, and odd
 * remainders, run one at a time.  lb_wave_autotune also tries two steps per
 * launch when allowed. */
int lb_wave_set_steps_per_launch(lb_wave *h, int32_t k);
int lb_wave_get_steps_per_launch(const lb_wave *h, int32_t *k);

/* Replay steady steps as captured HIP graphs of `chunk` steps (0 = off,
 * otherwise 2..4096).  A sequence is captured once per launch shape and
 * replayed at any step (the kernels read the step counter from the
 * workspace); steps where the measurement pipeline starts or an instance
 * stops are launched one by one.  Results are bit-identical either way. */
int lb_wave_set_graph(lb_wave *h, int32_t chunk);

/* Plain device-to-device copy of `bytes` (multiple of 16, 16-byte aligned
 * pointers) on `hip_stream`, asynchronous, with non-temporal loads and
 * stores.  A bandwidth reference for the step kernel's roofline: it moves
 * 2 * bytes through HBM with one read and one write stream. */
int lb_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *hip_stream);

/* ---- empty-cavity calibration of the driven standing wave ---- */

/* Runs the empty driven box (x sheets as above, no object; the field
 * depends on x only, so it is the three-population 1D lattice with rest
 * weight 1 - c0^2) for n_periods drive periods on the GPU, takes the
 * complex amplitude P(x) of rho1 at omega over the last n_fit periods, fits
 * |P|^2 = a + b cos 2kx + c sin 2kx with k the lattice wavenumber
 * (cos omega = 1 - c0^2 (1 - cos k)) and returns
 *   out[0] = A    = sqrt(a + sqrt(b^2 + c^2))  (rho1 amplitude at an antinode)
 *   out[1] = x_a  = the antinode closest to (nx-1)/2 from below
 *   out[2] = k
 *   out[3..5] = a, b, c
 * and, if host_P is not NULL, Re P(x), Im P(x) interleaved (2*nx doubles).
 * Needs lb_cavity_workspace_bytes(nx) bytes of device workspace; 16 <= nx <= 2048.
 * Synchronises the stream. */
size_t lb_cavity_workspace_bytes(int32_t nx);
int lb_cavity_calibrate(int32_t nx, double c0, double omega, double rho_a, double wall_phi,
                        int32_t n_periods, int32_t n_fit, void *dev_workspace,
                        size_t workspace_bytes, void *hip_stream, double *out, double *host_P);

/* The same calibration for callers that cannot allocate or pass device memory (harnesses that
 * forbid allocation, tight serving loops): no workspace argument, and no hipMalloc, hipFree or
 * other allocating call.  The kernel's lock-in sums go to a fixed array in the library's
 * device memory, 2 * 2048 doubles (32 KiB) per GPU, held until the process ends; nx above
 * 2048 is rejected with LB_EINVAL, like every other argument lb_cavity_calibrate rejects.
 * Results are those of lb_cavity_calibrate, bit for bit.  hip_stream must belong to the
 * current device.  Every call on one GPU uses that GPU's one array: calls that overlap on
 * the same GPU (other threads, or other streams before this call has returned) race.
 * Synchronises the stream. */
int lb_cavity_calibrate_noalloc(int32_t nx, double c0, double omega, double rho_a,
                                double wall_phi, int32_t n_periods, int32_t n_fit,
                                void *hip_stream, double *out, double *host_P);

#ifdef __cplusplus
}
#endif
#endif /* LB_WAVE_H */
