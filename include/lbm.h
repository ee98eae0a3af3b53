/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q19 lattice Boltzmann library.
 *
 * The library implements the fused pull iteration of Mawson & Revell,
 * "Memory transfer optimization for a lattice Boltzmann solver on Kepler
 * architecture nVidia GPUs" (Section 4.2, Algorithm 3): every fluid lattice
 * point gathers its 19 populations from x - e_i, applies the boundary rule,
 * forms rho and u (Eqs. (6)-(7)), the equilibrium (Eq. (5)) and the BGK
 * collision (Eqs. (2)-(3)), and stores the result in a second copy of the
 * population array (Section 4.1, footnote on the redundant copy).
 *
 * Conventions shared by every call:
 *   - Lattice point index: c = (z*ny + y)*nx + x, x fastest (Section 4.1).
 *     N = nx*ny*nz. Population i of point c is element i*N + c of a
 *     [19][N] array (structure of arrays, Section 4.1).
 *   - Velocity set: the 19 vectors of Eq. (4), in that order.
 *   - Flags (one byte per point): 0 = fluid, 1 = resting wall, 2 = moving
 *     wall, 3 = on-site velocity node at rest, 4 = on-site velocity node
 *     moving with u_wall. Values 1 and 2 are solid. Walls are halfway
 *     bounce-back: a fluid point whose neighbour x - e_i is solid takes the
 *     population it sent towards that wall, s_opp(i)(x), plus
 *     6 w_i (e_i . u_wall) for a moving wall (wall density 1). The box is
 *     periodic in x, y and z; walls come only from flags.
 *   - On-site velocity nodes (values 3, 4; the boundary type of the paper's
 *     cavity validation, Section 5) are fluid points on a box face, edge or
 *     corner whose solid neighbours are exactly the cells beyond one to three
 *     axis-aligned walls. After the gather, the populations that would come
 *     from solid cells are rebuilt so that the node carries its prescribed
 *     velocity and a density fixed by mass balance: an unknown population
 *     whose opposite is known takes that opposite plus 6 w_i e_i . j plus a
 *     transverse correction (j = rho u - F/2), and a pair of opposite
 *     unknowns (edges, corners) takes the equilibrium at (rho, u). The
 *     prescribed velocity is u_wall for value 4 and zero for value 3; the
 *     macroscopic output reports it exactly (up to rounding).
 *   - Body force (optional): Guo forcing, u = (m + F/2)/rho and source
 *     (1 - 1/(2 tau)) w_i [3(e_i - u) + 9 (e_i . u) e_i] . F.
 *   - The state is the array of post-collision populations. Values stored
 *     at solid points are unspecified (no fluid point reads them; the
 *     macroscopic output reports rho = 0, u = 0 there).
 *   - Pointers named *_dev are device pointers (HIP global memory on the
 *     lattice's device); pointers named *_host are host memory. Vector
 *     fields are [3][N] float, component slowest.
 *   - Every call that takes device pointers enqueues its work on the
 *     lattice's HIP stream and returns before the GPU finishes, unless
 *     stated otherwise. The caller keeps device buffers alive until the
 *     stream has passed the work.
 *   - Errors are status codes; no call throws. A failed HIP call makes the
 *     lattice's error sticky: every later call on it returns
 *     LBM_ERR_DEVICE (LBM_ERR_STATE for lbm_step). lbm_last_error() gives
 *     a message for the calling thread's last failure.
 *   - One lattice must not be used from two host threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,   /* bad argument; nothing was changed */
    LBM_ERR_OOM = 2,       /* device or host allocation failed */
    LBM_ERR_DEVICE = 3,    /* a HIP call failed; the lattice is now unusable */
    LBM_ERR_STATE = 4,     /* call not valid in the lattice's current state */
    LBM_ERR_NONFINITE = 5  /* a finite-value check found NaN or Inf */
} lbm_status;

/* Population storage in HBM. Arithmetic is always FP32. The 16-bit forms
 * store the offset f_i - w_i rounded to nearest even. */
typedef enum lbm_storage {
    LBM_STORAGE_F32 = 0,
    LBM_STORAGE_F16 = 1,   /* IEEE binary16 offsets */
    LBM_STORAGE_BF16 = 2   /* bfloat16 offsets */
} lbm_storage;

/* AB: two population arrays, swapped after every step (Section 4.1).
 * AA: one array updated in place by alternating a gather/scatter step and a
 *     local step (each work-item reads and writes the same 19 slots). */
typedef enum lbm_pattern {
    LBM_PATTERN_AB = 0,
    LBM_PATTERN_AA = 1
} lbm_pattern;

typedef struct lbm_options {
    int storage;          /* lbm_storage */
    int pattern;          /* lbm_pattern */
    void* hip_stream;     /* hipStream_t to launch on; NULL = the null stream */
    int block_x;          /* work-group shape for the step kernels; 0 = default */
    int block_y;          /*   (block_x * block_y <= 1024, block_x >= 1) */
    int timing_capacity;  /* > 0: record a HIP event after every step (ring of
                             this many) for lbm_step_times */
    int check_interval;   /* > 0: lbm_step checks for non-finite values every
                             this many steps (synchronises the stream) */
    int device;           /* HIP device ordinal; -1 = the current device */
    int cells_per_lane;   /* AB step: points per work-item. 0 = automatic (8
                             for 16-bit storage when nx % 8 == 0 and either
                             nx >= 256 or at least 8% of the fluid points have
                             a solid neighbour, else 4 when nx % 4 == 0,
                             else 1; 1 for lattices of at most 2^18 points
                             without solid points; bfloat16 steps taken while
                             a body force is set use 4 where the automatic
                             choice is 8);
                             1; 4; or 8 (16-bit storage only: 16-byte
                             accesses). 4 and 8 need
                             nx to be a multiple of them and
                             block_x * block_y <= 256 (block_x then counts
                             work-items) */
    int gather_mode;      /* FP32 multi-point AB step: 0 = automatic (early
                             gather when at least 8% of the fluid points have a
                             solid neighbour), 1 = flags first, 2 = early
                             gather (the 19 loads are issued before the point
                             flags are examined). Results are identical. */
    int groups_per_cu;    /* multi-point AB step: work-groups resident per
                             compute unit. 0 = automatic (8 for FP32 storage
                             with the default work-group shape when the flags
                             come first, else as many as the registers allow),
                             -1 = as many as the registers allow, 1..64 = that
                             cap (LDS is reserved per work-group, never used).
                             Results are identical. */
    void* population_dev[2]; /* optional caller-owned device buffers for the
                             population arrays: both NULL = the library
                             allocates them; otherwise the AB pattern needs
                             both and AA the first, each of at least
                             lbm_buffer_sizes().population_bytes, 256-byte
                             aligned, not overlapping, alive and unused by
                             the caller until lbm_destroy returns. The
                             library never frees them and lbm_device_bytes
                             does not count them. */
} lbm_options;

/* Device memory a lattice of the given size and options needs (Section 4.1:
 * 19 populations per point). population_bytes: one population array (the AB
 * pattern uses two, AA one); adjoint_bytes: the workspace of lbm_adjoint
 * (two adjoint arrays and per-work-group partial sums); state_bytes: one FP32
 * state [19][N], the unit of the checkpoint store. */
typedef struct lbm_buffer_sizes {
    size_t population_bytes;
    int population_arrays;
    size_t adjoint_bytes;
    size_t state_bytes;
} lbm_buffer_sizes;

typedef struct lbm_lattice lbm_lattice;

/* Fills *opt with the defaults: F32, AB, null stream, default block shape,
 * no timing, no checks, current device. */
void lbm_options_default(lbm_options* opt);

/*
 * Creates a lattice of nx*ny*nz points with relaxation time tau (Eq. (2)),
 * at rest (rho = 1, u = 0: f_i = w_i). flags_host: N bytes in index order,
 * or NULL for all fluid; copied, so the caller may free it on return.
 * Errors: LBM_ERR_INVALID if any n <= 0, N >= 2^30, tau <= 0.5 or not
 * finite, a flag value > 4, or out == NULL (checked before any HIP call),
 * and for an on-site node whose solid neighbours do not form a box face,
 * edge or corner (found on the device during creation); LBM_ERR_OOM;
 * LBM_ERR_DEVICE.
 */
lbm_status lbm_create(int nx, int ny, int nz, float tau, const uint8_t* flags_host,
                      lbm_lattice** out);

/* As lbm_create with explicit options (opt == NULL: defaults). Errors as
 * lbm_create, plus LBM_ERR_INVALID for an unknown storage/pattern or a bad
 * block shape. */
lbm_status lbm_create_ex(int nx, int ny, int nz, float tau, const uint8_t* flags_host,
                         const lbm_options* opt, lbm_lattice** out);

/* Releases everything the library allocated for the lattice (after waiting
 * for its stream). NULL is a no-op. Caller-owned buffers (population_dev,
 * lbm_set_trajectory_buffer, lbm_set_adjoint_buffer) are not freed; they may
 * be released once this returns. */
void lbm_destroy(lbm_lattice* lat);

/* Sizes of the device buffers a lattice of nx*ny*nz points created with
 * `opt` (NULL: defaults) uses, so that a caller can allocate them itself
 * (population_dev in lbm_options, lbm_set_adjoint_buffer). Nothing is
 * allocated. Errors: LBM_ERR_INVALID for the arguments lbm_create_ex rejects
 * before touching the device. */
lbm_status lbm_query_buffer_sizes(int nx, int ny, int nz, const lbm_options* opt, lbm_buffer_sizes* out);

/* Bytes of the checkpoint store lbm_forward_checkpointed(T, K) uses on a
 * lattice of nx*ny*nz points: ceil(T/K) checkpoints plus min(K, T) - 1
 * recomputed states (at least one checkpoint), each state_bytes. 0 for
 * invalid arguments. */
size_t lbm_trajectory_bytes(int nx, int ny, int nz, int T, int K);

/* Gives the lattice a caller-owned device buffer for the checkpoint store of
 * lbm_forward_checkpointed (`bytes` long, 256-byte aligned). Later rollouts
 * whose lbm_trajectory_bytes exceeds `bytes` fail with LBM_ERR_INVALID instead
 * of allocating. NULL returns to library-allocated storage. Drops a recorded
 * trajectory. The buffer must stay alive and untouched by the caller until
 * it is replaced or the lattice is destroyed. */
lbm_status lbm_set_trajectory_buffer(lbm_lattice* lat, void* dev, size_t bytes);

/* Gives the lattice a caller-owned device workspace for lbm_adjoint of at
 * least lbm_buffer_sizes().adjoint_bytes (256-byte aligned); NULL returns to
 * library-allocated storage (allocated at the first lbm_adjoint). The buffer
 * must stay alive and untouched by the caller until it is replaced or the
 * lattice is destroyed. Errors: LBM_ERR_INVALID if `bytes` is too small or
 * the pointer misaligned. */
lbm_status lbm_set_adjoint_buffer(lbm_lattice* lat, void* dev, size_t bytes);

/* Lattice sizes and storage, for the caller's bookkeeping. */
lbm_status lbm_get_info(const lbm_lattice* lat, int* nx, int* ny, int* nz, int* storage,
                        int* pattern);

/* Changes the stream later work is launched on (NULL = null stream). Work
 * already enqueued on the previous stream is ordered before later work on the
 * new one (an event recorded on the old stream is waited for on the new one;
 * the host does not block). */
lbm_status lbm_set_stream(lbm_lattice* lat, void* hip_stream);

/* Name of the device kernel the next lbm_step launches (the fused step of
 * Algorithm 3 in the variant the lattice's storage, pattern, parity, force
 * and geometry select), as the HIP runtime reports it, demangled; written to
 * buf (NUL-terminated, truncated to cap bytes). For measurement tools that
 * match it against profiler traces. Errors: LBM_ERR_INVALID for a NULL or
 * empty buffer. */
lbm_status lbm_step_kernel_name(lbm_lattice* lat, char* buf, size_t cap);

/* Relaxation time (Eq. (2)); tau > 0.5. Invalidates a recorded trajectory. */
lbm_status lbm_set_tau(lbm_lattice* lat, float tau);

/* Velocity of all flag-2 points and of the flag-4 on-site nodes (Section 5
 * uses a moving lid). Each component must be finite and |u| < 0.3
 * (low-Mach guard). */
lbm_status lbm_set_wall_velocity(lbm_lattice* lat, float ux, float uy, float uz);

/* Uniform body force (Guo forcing); clears a force field. Invalidates a
 * recorded trajectory. */
lbm_status lbm_set_force_uniform(lbm_lattice* lat, float fx, float fy, float fz);

/* Per-point body force F_dev: [3][N] float on the device, copied into the
 * lattice (the caller's buffer may be freed once the stream has passed the
 * copy). NULL removes the field (force becomes zero). Invalidates a
 * recorded trajectory. */
lbm_status lbm_set_force_field(lbm_lattice* lat, const float* F_dev);

/* f = f^eq(rho, u) at every point (Eq. (5)); rho_dev [N] or NULL (rho = 1),
 * u_dev [3][N] or NULL (u = 0). */
lbm_status lbm_init_equilibrium(lbm_lattice* lat, const float* rho_dev, const float* u_dev);

/* Enqueues n fused pull steps (Algorithm 3). n = 0 is a no-op.
 * Errors: LBM_ERR_INVALID for n < 0; LBM_ERR_STATE after a device error;
 * LBM_ERR_NONFINITE when a due check (check_interval) finds NaN/Inf. */
lbm_status lbm_step(lbm_lattice* lat, int n);

/* n >= 1 steps as lbm_step, where the last one also writes its in-step
 * rho and u = (sum_i e_i p_i + F/2)/rho (Eqs. (6)-(7)) into rho_dev [N] and
 * u_dev [3][N] (0 at solid points): the four extra stores per point of the
 * paper's macroscopic-output variant (Section 4.1), fused into the step
 * instead of a separate pass. These equal lbm_macros of the resulting state
 * up to rounding. In the AA pattern the output is a separate pass after the
 * steps. Errors: as lbm_step; LBM_ERR_INVALID for n < 1 or a NULL output. */
lbm_status lbm_step_macros(lbm_lattice* lat, int n, float* rho_dev, float* u_dev);

/* Writes rho = sum_i s_i and u = (sum_i e_i s_i - F/2)/rho (Eqs. (6)-(7) on
 * the post-collision state) into rho_dev [N] and u_dev [3][N]; solid points
 * get rho = 0, u = 0. Either pointer may be NULL to skip it, not both. */
lbm_status lbm_macros(lbm_lattice* lat, float* rho_dev, float* u_dev);

/* Copies the state out as plain populations f_dev [19][N] float in the
 * structure-of-arrays order of Section 4.1 (element i*N + c; offsets added
 * back, the AA layout resolved, whatever the internal plane layout).
 * Errors: LBM_ERR_INVALID for NULL. */
lbm_status lbm_get_populations(lbm_lattice* lat, float* f_dev);

/* Replaces the state with f_dev [19][N] float, plain populations in the order
 * of lbm_get_populations (16-bit storage rounds the offsets to nearest even).
 * Invalidates a recorded trajectory. Errors: LBM_ERR_INVALID for NULL. */
lbm_status lbm_set_populations(lbm_lattice* lat, const float* f_dev);

/* Test hook: n steps of the streaming half of Algorithm 3 alone (the pull of
 * Section 4.2 with bounce-back at solid neighbours, no collision and no
 * moving-wall term): an exact permutation of the stored values. On-site
 * nodes stream like plain fluid points here. Errors: LBM_ERR_INVALID for
 * n < 0. */
lbm_status lbm_debug_stream_only(lbm_lattice* lat, int n);

/*
 * Runs T steps from the current state and keeps the states at steps 0, K,
 * 2K, ... in device memory for lbm_adjoint (checkpoint-every-K). A last
 * segment shorter than K is allowed. F32 storage, the AB pattern and
 * lattices without on-site nodes only.
 * Errors: LBM_ERR_INVALID (T < 0, K <= 0); LBM_ERR_STATE (on-site nodes, other storage or
 * pattern); LBM_ERR_OOM.
 */
lbm_status lbm_forward_checkpointed(lbm_lattice* lat, int T, int K);

/*
 * Discrete adjoint of the rollout recorded by lbm_forward_checkpointed.
 * dL_du_dev: [3][N] gradient of a scalar loss with respect to u(T) as
 * returned by lbm_macros (values at solid points are ignored). Writes
 * grad_F_dev [3][N] = dL/dF (overwritten; zero at solid points) and
 * *grad_tau_host = dL/dtau. Recomputes each segment from its checkpoint,
 * then runs the reverse step for every time step of the segment.
 * Synchronises the stream before returning (grad_tau is a host value).
 * Errors: LBM_ERR_STATE without a valid trajectory (parameters, state or
 * force changed since it was recorded); LBM_ERR_INVALID; LBM_ERR_OOM.
 */
lbm_status lbm_adjoint(lbm_lattice* lat, const float* dL_du_dev, float* grad_F_dev,
                       double* grad_tau_host);

/*
 * The same reverse sweep as lbm_adjoint, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): it calls no allocating routine. Its two
 * adjoint arrays, per-work-group dL/dtau partials and their sum live in one
 * static device array of the library (40 MiB per GPU, held until the process
 * ends), so the lattice may have at most 2^18 points (e.g. 64^3); larger
 * lattices get LBM_ERR_INVALID and use lbm_adjoint. The trajectory must come
 * from lbm_forward_checkpointed (its store allocated then, or given with
 * lbm_set_trajectory_buffer). Results are bit-identical to lbm_adjoint
 * (dL/dtau is summed in the same order). Every call on one GPU shares that
 * array: calls that overlap on the same GPU (two streams, two threads) race
 * and give wrong results. Synchronises the stream before returning.
 * Errors: as lbm_adjoint; LBM_ERR_INVALID for more than 2^18 points.
 */
lbm_status lbm_adjoint_noalloc(lbm_lattice* lat, const float* dL_du_dev, float* grad_F_dev,
                               double* grad_tau_host);

/* Checks every stored population of the fluid points for NaN/Inf.
 * Synchronises. Returns LBM_OK or LBM_ERR_NONFINITE. */
lbm_status lbm_check_finite(lbm_lattice* lat);

/* Per-step durations (ms) of the most recent steps recorded with
 * timing_capacity > 0, oldest first: at most cap values into ms_host,
 * *count = number written. This is the iteration-time series whose spread
 * and periodic components Section 6 (Table 5) analyses. Synchronises.
 * Clears the log. Errors: LBM_ERR_STATE without a timing log;
 * LBM_ERR_INVALID for bad output arguments. */
lbm_status lbm_step_times(lbm_lattice* lat, float* ms_host, int cap, int* count);

/* Waits for all work enqueued on the lattice's stream. */
lbm_status lbm_sync(lbm_lattice* lat);

/* Device bytes the library holds for this lattice. */
size_t lbm_device_bytes(const lbm_lattice* lat);

/* Static name of a status value. */
const char* lbm_status_string(lbm_status st);

/* Message of the calling thread's last failed call ("" if none). */
const char* lbm_last_error(void);

/*
 * Bandwidth probe used to state the measured copy ceiling of the device
 * (the paper quotes measured rather than nominal bandwidth, Section 2.2):
 * dst[k] = src[k] for k < n floats (device pointers, 16-byte aligned, not
 * overlapping), on the given stream: one 16-byte chunk per work-item with
 * non-temporal loads and stores, like the vector step's accesses.
 * LBM_ERR_INVALID for a NULL or misaligned pointer with n > 0.
 */
lbm_status lbm_copy_f32(const float* src_dev, float* dst_dev, size_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
