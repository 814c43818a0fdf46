/*
 * ljsde.h -- C ABI of the MI355X (gfx950) RL-JSDE reconstruction library.
 *
 * RL-JSDE reconstructs an image on a grid of twice the sensor resolution from
 * three-quarter-sampling measurements (Sec. II, eq. (1)): every sensor pixel
 * integrates the three transparent quadrants of its 2x2 footprint; the fourth
 * (the opaque quadrant) is given per pixel by a recurrent pattern. Every
 * B x B target block is modelled on its surrounding W x W window by a sparse
 * Fourier model built one coefficient at a time (Sec. III; Sec. IV eqs.
 * (11)-(18)); only the central block of each window is written out.
 *
 * Conventions shared by all entry points
 *  - Return value: 0 (LJSDE_OK) on success, a negative LJSDE_E* code on
 *    failure. ljsde_last_error() then describes the failure; the text is
 *    thread-local and valid until the next call from the same thread.
 *  - Images are row-major [row][col]. A sensor image of R x C pixels yields a
 *    reconstruction of 2R x 2C pixels.
 *  - Pattern codes: o = 2*a + b in {0,1,2,3}, where (a, b) is the (row, col)
 *    position of the opaque quadrant inside the 2x2 footprint. Sensor pixel
 *    (i, j) uses pattern[(i % pat_rows) * pat_cols + (j % pat_cols)].
 *  - Device pointers are HIP device addresses on the current device; the
 *    caller owns them and keeps them alive until the stream work completes.
 *    `stream` is a hipStream_t (NULL = the default stream). Reconstruction
 *    calls are asynchronous; errors raised by a running kernel surface at the
 *    next call or at ljsde_synchronize().
 *  - The library owns its plan tables until ljsde_release(); it never frees
 *    or synchronises caller memory.
 *  - All entry points are safe to call from several host threads; calls that
 *    use the same plan on different streams may run concurrently.
 */
#ifndef LJSDE_H
#define LJSDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
    LJSDE_OK = 0,
    LJSDE_EINVAL = -1,       /* invalid argument (checked on the host, before any GPU work) */
    LJSDE_EUNSUPPORTED = -2, /* valid for the method, but no kernel for this shape */
    LJSDE_ENOMEM = -3,       /* host or device allocation failed */
    LJSDE_EHIP = -4,         /* HIP runtime error, including "no device" */
    LJSDE_EBADID = -5        /* unknown or released pattern id */
};

/* plan flags */
enum {
    LJSDE_FP64 = 1,           /* FP64 everywhere: measurements/out are double */
    LJSDE_FP32 = 2,           /* FP32 projections, metric and argmax search; FP64 loop state,
                                 tables, step and energy; an FP32 near tie (relative 1e-4) is
                                 re-decided in FP64. out is float; measurements are float,
                                 or double with LJSDE_INPUT_F64 */
    LJSDE_DFT_SPLITBF16 = 4,  /* FP32 plans, W = 32: window DFT on MFMA with 3-term split-BF16
                                 products and FP32 accumulation instead of FP64 MFMA (relative
                                 error ~2^-16 in the initial state; selections can then
                                 diverge from FP64 at near ties). With LJSDE_STATE_FP32 also */
    LJSDE_Q_ONES = 8,         /* frequency weight q = 1 (test mode) */
    LJSDE_STATE_FP32 = 16,    /* FP32 plans: keep the loop state and its updates in FP32 too
                                 (no FP64 re-decision); greedy selections can then diverge
                                 from FP64 at near ties */
    LJSDE_DENSE_C = 32,       /* the dense form of Sec. IV, FP64 arithmetic. Per class the full
                                 W^2 x W^2 matrix C of eq. (14) is built in device memory
                                 (16 MiB per class at W = 32, on the first reconstruction of an
                                 image size; LJSDE_ENOMEM if it does not fit), each window
                                 keeps R of eq. (12) for all W^2 frequencies and subtracts a
                                 column of C per iteration (eq. (17)). Same results as the
                                 factorised FP64 path; single images and batches. With
                                 LJSDE_FP32 the output is float (and the measurements unless
                                 LJSDE_INPUT_F64; the arithmetic stays FP64); not with
                                 LJSDE_DFT_SPLITBF16 or
                                 LJSDE_STATE_FP32 */
    LJSDE_WEIGHTS = 64,       /* reported by ljsde_plan_info for plans made by
                                 ljsde_plan_weights (ignored there, refused by ljsde_plan) */
    LJSDE_INPUT_F64 = 128,    /* FP32 plans: the measurements are double (the output stays
                                 float). The kernels widen every measurement to FP64 on load,
                                 so an FP32 plan then sees exactly the input an FP64 plan sees.
                                 Implied by LJSDE_FP64 */
    LJSDE_PLAIN_L = 4096      /* plain L-JSDE (Sec. III; Sec. IV eqs. (4)-(10), (15),
                                 (16)), the method the recurrent form accelerates. Each window
                                 keeps its residual in the measurement domain and evaluates the
                                 numerator of eq. (10) for every basis function in every
                                 iteration: a product with the dense (W/2)^2 x W^2 matrix of basis
                                 responses a_m(f) = sum A_m Phi_f, O(W^4) per iteration. The
                                 responses of every local measurement matrix of an image size are
                                 built in device memory on its first reconstruction (16 B x
                                 (W/2)^2 x W^2 per class: 4 MiB at W = 32; LJSDE_ENOMEM if they
                                 do not fit). Same results as the recurrent form. FP64 arithmetic;
                                 with LJSDE_FP32 the output is float (and the measurements unless
                                 LJSDE_INPUT_F64). Single-image calls only; not with
                                 LJSDE_DENSE_C, LJSDE_DFT_SPLITBF16 or LJSDE_STATE_FP32. Every
                                 pixel shape and ljsde_plan_weights layouts */
};

/*
 * Pixel shape (Sec. I; Sec. II eq. (1): any such layout is a measurement
 * matrix). Flag bits 8..11 hold a mask of quadrant offsets d: the sensor
 * pixel of code o collects light on the quadrants o XOR d (quadrant index
 * 2 * row + column inside its 2x2 footprint) for the bits d that are set.
 * 0 means three-quarter sampling (0xE: L-shaped pixels, the code names the
 * opaque quadrant); 0x1 is quarter sampling (the code names the one
 * transparent quadrant). The other masks with three or one bits are the same
 * two layouts with relabelled codes and run on the same kernels (class
 * tables then report the relabelled codes). Masks with two bits (half and
 * diagonal pixels) or four (full pixels) run as their 0/1 quadrant weights on
 * the general-layout dense form (see ljsde_plan_weights): they need
 * LJSDE_DENSE_C (or LJSDE_PLAIN_L), else LJSDE_EUNSUPPORTED, and ljsde_plan_info
 * reports LJSDE_WEIGHTS for them. LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32
 * exist for three-quarter sampling only.
 * Frequencies that no measurement of a window responds to (D of eq. (13) at
 * most 1e-13 of the window's largest D: e.g. rho = W/2 for side-by-side
 * quadrant pairs) are never selected.
 */
#define LJSDE_SHAPE(mask) ((((unsigned)(mask)) & 15u) << 8)
enum {
    LJSDE_SHAPE_THREE_QUARTER = 0xE00,
    LJSDE_SHAPE_QUARTER = 0x100
};

/*
 * ljsde_plan -- validate and register a reconstruction plan.
 *
 * Defines the local measurement matrices of a recurrent three-quarter (or
 * quarter) sampling sensor (Sec. II, Sec. IV: all windows with the same local
 * measurement matrix share their precomputed tables).
 *  pattern   host, pat_rows x pat_cols uint8 codes (copied; the caller keeps
 *            ownership). A non-recurrent sensor passes the whole sensor.
 *  window    W, model window side in high-resolution pixels (Sec. III);
 *            even, (W - B) divisible by 4. Kernels exist for W in {16, 32}.
 *  block     B, target block side (Sec. III); even; kernels exist for B in
 *            {4, 8} with B <= W.
 *  iters     nu_max >= 1, model-generation iterations per window (Sec. IV).
 *  rho       spatial weight base of w_m = rho^d (eq. (8)), 0 < rho <= 1.
 *  gamma     orthogonality deficiency compensation gamma_odc of eq. (15),
 *            0 < gamma < 2.
 *  flags     exactly one of LJSDE_FP64 / LJSDE_FP32, plus options and an
 *            optional pixel shape (LJSDE_SHAPE_*).
 * Returns a pattern id >= 0, or a negative status. Needs no GPU: tables for
 * an image size are built and uploaded on its first reconstruction.
 */
int ljsde_plan(const uint8_t *pattern, int pat_rows, int pat_cols,
               int window, int block, int iters, double rho, double gamma,
               unsigned flags);

/*
 * ljsde_plan_weights -- validate and register a plan for a general layout of
 * the 2x2-footprint sensor (Sec. II, eq. (1): every measurement is a weighted
 * sum of the high-resolution pixels under its sensor pixel; Sec. I: RL-JSDE
 * applies to any recurrent layout). Sensor pixel (i, j) weighs quadrant
 * q = 2*a + b of its footprint (row 2i + a, column 2j + b of the
 * reconstruction) by weights[((i % pat_rows) * pat_cols + (j % pat_cols)) * 4 + q].
 *  weights   host, pat_rows x pat_cols x 4 finite doubles (copied; the
 *            caller keeps ownership). 0/1 weights of a pixel shape give that
 *            shape's measurement matrix.
 *  window, block, iters, rho, gamma  as for ljsde_plan.
 *  flags     LJSDE_DENSE_C with LJSDE_FP64 (double measurements and output)
 *            or LJSDE_FP32 (float output, and float measurements unless
 *            LJSDE_INPUT_F64; FP64 arithmetic either way), or LJSDE_PLAIN_L
 *            with either; optionally LJSDE_Q_ONES; no pixel shape.
 *            Without LJSDE_DENSE_C or LJSDE_PLAIN_L -> LJSDE_EUNSUPPORTED.
 * Per class the tables hold the ten spectra S_qq' = DFT(w A_q A_q') (q <= q')
 * and the per-pixel weights; C of eq. (14) is built from them on the device.
 * Frequencies that leave no trace in a window (D of eq. (13) is 0 in exact
 * arithmetic, e.g. equal weights on all four quadrants at sigma = W/2; in
 * FP64 at most 1e-13 of the window's largest D) are never selected. A
 * window whose weights are all 0 observes no frequency: every iteration picks
 * frequency 0 with a zero step, and its block of the output is 0.
 * Returns a pattern id >= 0, or a negative status. Needs no GPU.
 */
int ljsde_plan_weights(const double *weights, int pat_rows, int pat_cols,
                       int window, int block, int iters, double rho, double gamma,
                       unsigned flags);

/*
 * ljsde_set_energy_floor -- optional stopping test (Sec. IV: iterate up to
 * nu_max). A window stops early once its weighted residual energy (eq. (8)),
 * tracked in FP64, falls to tau times its initial value. tau = 0 (default)
 * disables the test. 0 <= tau < 1.
 */
int ljsde_set_energy_floor(int pattern_id, double tau);

/*
 * ljsde_reconstruct -- reconstruct one image (Sec. IV eqs. (11)-(18) per
 * target block).
 *  measurements  device, sensor_rows x sensor_cols, double (FP64 plans and
 *                FP32 plans with LJSDE_INPUT_F64) or float (other FP32
 *                plans). Sides must be multiples of B/2.
 *  out           device, (2*sensor_rows) x (2*sensor_cols), double (FP64
 *                plans) or float (FP32 plans); every pixel is written.
 *  stream        hipStream_t or NULL.
 * Both buffers must be device (or managed) memory of the current device: a
 * host pointer is LJSDE_EINVAL, and nothing is launched.
 * FP64 plans run one launch with one wavefront per window; FP32 plans run
 * the persistent batched kernel with a batch of one.
 */
int ljsde_reconstruct(const void *measurements, int sensor_rows, int sensor_cols,
                      int pattern_id, void *out, void *stream);

/*
 * ljsde_reconstruct_diag -- as ljsde_reconstruct, and also records the
 * selected frequency sigma*W + rho of every iteration (eq. (11)).
 *  selections  device int16, [n_windows][iters] with windows in row-major
 *              block order (n_windows = (2R/B) * (2C/B)); entries after an
 *              early stop are -1.
 */
int ljsde_reconstruct_diag(const void *measurements, int sensor_rows, int sensor_cols,
                           int pattern_id, void *out, int16_t *selections, void *stream);

/* one image of a batch */
typedef struct {
    const void *measurements; /* device, as for ljsde_reconstruct (double or float by the
                                 job's plan: jobs of one batch may differ) */
    int sensor_rows;
    int sensor_cols;
    int pattern_id;           /* see ljsde_reconstruct_batch for the plans one batch may mix */
    void *out;                /* device */
} ljsde_job;

/*
 * ljsde_reconstruct_batch -- reconstruct many images of uneven size and
 * pattern in one launch (device state per batch shape and stream, kept until
 * a plan of the batch is released; launches on different streams may
 * overlap). Two kinds of batch, by the first job's plan:
 *  - FP32 plans of the factorised form: one persistent launch, captured once
 *    as a HIP graph per batch shape and stream and replayed afterwards. All
 *    plans need equal window, block, iterations, rho, gamma, energy floor,
 *    state precision, DFT mode and pixel shape (LJSDE_EINVAL otherwise).
 *  - plans of the dense form (LJSDE_DENSE_C, FP64 or FP32): one launch over
 *    the windows of all images, each image with its own dense C (built on
 *    the first use of its plan and size). All plans need the dense form and
 *    equal window, block, iterations, rho, gamma, energy floor, pixel shape
 *    and precision (LJSDE_EINVAL otherwise).
 * Other plans (FP64 factorised, LJSDE_PLAIN_L) -> LJSDE_EUNSUPPORTED.
 * `jobs` is host memory, read during the call only; an empty batch is
 * LJSDE_EINVAL, and so is a job whose measurements or out are not device
 * memory (checked whenever a job's buffers change; nothing is launched then).
 */
int ljsde_reconstruct_batch(const ljsde_job *jobs, int n_jobs, void *stream);

/*
 * ljsde_reconstruct_noalloc -- ljsde_reconstruct for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). It runs the same persistent FP32 kernel
 * as ljsde_reconstruct with a batch of one, with the same results; its work
 * memory (work counters, the job and the list of window groups) is a static
 * device array of the library, one per GPU, held until the process ends.
 *  measurements, sensor_rows, sensor_cols, pattern_id, out, stream
 *            as for ljsde_reconstruct. FP32 plans of the factorised form
 *            only (LJSDE_FP64, LJSDE_DENSE_C, LJSDE_STATE_FP32 and
 *            LJSDE_PLAIN_L plans -> LJSDE_EUNSUPPORTED).
 * Precondition: the plan has already reconstructed an image of this sensor
 * size on this device (ljsde_reconstruct, ljsde_reconstruct_batch or
 * ljsde_reconstruct_diag build and upload its class tables); otherwise
 * LJSDE_EINVAL, and nothing runs.
 * Limit: the work list holds at most 262144 groups (6 MiB). A group holds up
 * to 4 windows of one local measurement matrix (4 by default, or the width
 * ljsde_autotune chose for that shape: 1, 2 or 4), so images of more than
 * 1048576 target blocks (e.g. beyond 4096 x 4096 output pixels at B = 4), and
 * smaller ones whose list exceeds the limit, are LJSDE_EINVAL.
 * The call makes no device allocation or free. It builds its host-side work
 * list once per plan, image size and group width (host memory, kept with the
 * plan) and uploads it only when that changes since the device's last call.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.
 */
int ljsde_reconstruct_noalloc(const void *measurements, int sensor_rows, int sensor_cols,
                              int pattern_id, void *out, void *stream);

/*
 * ljsde_autotune -- time the launch variants of the persistent kernel on this
 * batch and keep the fastest for later batch calls of the same shape class:
 * windows per workgroup (1, 2, 4), resident workgroups per compute unit (the
 * maximum or one fewer), window groups taken per work claim (1, 2, 4), and,
 * for W = 32 without split-BF16, the LDS layout (per-lane q/D and twiddles
 * re-read from LDS every iteration, or held in registers) and the DFT tile
 * shape (the window DFT on FP64 MFMA 16x16x4 tiles, or as FP64 VALU row and
 * column passes, which sums in another order: outputs equal up to FP64
 * rounding). The search is staged: the first two knobs, then the claim
 * size, then the last two, each from the best so far. Results are cached in
 * memory and, if LJSDE_TUNE_CACHE names a file, in that JSON file ("key" :
 * [windows per workgroup, groups per claim, fewer workgroups, q/D in
 * registers, VALU DFT]). Synchronises `stream`. Outputs of the batch are
 * overwritten. For tests, LJSDE_VARIANT="nw,chunk,fewer,qreg,vdft" in the
 * environment forces the variant of batch states created afterwards.
 */
int ljsde_autotune(const ljsde_job *jobs, int n_jobs, void *stream);

/* ljsde_synchronize -- wait for `stream`; reports pending HIP errors. */
int ljsde_synchronize(void *stream);

/* ljsde_release -- free a plan's tables; later use of the id -> LJSDE_EBADID. */
int ljsde_release(int pattern_id);

/* ljsde_last_error -- text of the last failure on this thread ("" if none). */
const char *ljsde_last_error(void);

/*
 * Host-side introspection (no GPU needed).
 *
 * ljsde_class_count -- number of distinct local measurement matrices (Sec.
 * IV: B, C and D are shared by all windows with the same one) for an image
 * of sensor_rows x sensor_cols, and the class of every window:
 *  class_of_window  host int32 [n_windows] in row-major block order, or NULL.
 * Returns the class count (>= 1) or a negative status.
 */
int ljsde_class_count(int pattern_id, int sensor_rows, int sensor_cols,
                      int32_t *class_of_window);

/*
 * ljsde_class_tables -- the FP64 tables of one class, as used on the GPU.
 *  S      host double [Ws*Ws][4][2] or NULL: weighted-mask spectra
 *         S_o(k, l) = sum over the class's present sensor pixels (i', j') with
 *         code o of w(i', j') exp(-2 pi i (i' k + j' l) / Ws), Ws = W/2
 *         (the factorised form of C, eq. (14)); index [k*Ws + l][o][re, im].
 *         Plans of ljsde_plan_weights: [Ws*Ws][10][2], the spectra of
 *         w(i', j') A(i', j', q) A(i', j', q') for the pairs q <= q' in the
 *         order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).
 *  D      host double [W*W] or NULL: the normaliser of eq. (13).
 *  codes  host int8 [Ws*Ws] or NULL: pattern code per local sensor pixel,
 *         -1 where the pixel lies outside the image (0 inside for plans of
 *         ljsde_plan_weights).
 */
int ljsde_class_tables(int pattern_id, int sensor_rows, int sensor_cols, int class_index,
                       double *S, double *D, int8_t *codes);

/*
 * ljsde_plan_info -- the geometry of a plan (any output pointer may be NULL):
 * window W, block B, iterations nu_max and the flags it was created with.
 */
int ljsde_plan_info(int pattern_id, int *window, int *block, int *iters, unsigned *flags);

/* ljsde_version -- ABI version (major * 10000 + minor * 100 + patch). */
int ljsde_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LJSDE_H */
