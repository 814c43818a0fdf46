// Shared host/device declarations of the RL-JSDE library (not part of the ABI).
#pragma once

#include <cstddef>
#include <cstdint>

namespace ljsde {

// Class-independent constants, FP64, on the device.
struct DevConsts {
    const double *w;    // [Ws*Ws] spatial weights w_m = rho^d_m (eq. (8))
    const double *ew;   // [W][2]  exp(+i 2 pi k / W), k < W
    const double *dft;  // [Ws][2] exp(-i 2 pi k / Ws), k < Ws
    const double *H;    // [W*W][4][2] H_o(sigma, rho): response of the pixel of code o
                        // (its shape's quadrants) to the basis function (sigma, rho)
    const double *q;    // [W*W]   frequency weight q of eqs. (10)-(11)
};

// KParams::shape of a plan with general per-pixel quadrant weights (Sec. II,
// eq. (1): any 2x2-footprint layout), outside the range of the 4-bit masks.
constexpr int SHAPE_GENERAL = 0x10;

// Byte offsets inside one class block of the device table.
struct ClassLayout {
    int offS;      // double [Ws*Ws][4][2]  S_o(k, l); general layouts: [Ws*Ws][10][2]
                   //                        S_qq'(k, l) for q <= q'
    int offQD64;   // double [W*W]          q / D   (0 where D <= 0)
    int offInvD;   // double [W*W]          1 / D   (0 where D <= 0)
    int offQD32;   // float  [W*W]          q / D
    int offCodes;  // int8   [Ws*Ws]        code, -1 outside the image (general layouts: 0)
    int offA;      // double [Ws*Ws][4]     quadrant weights per pixel (general layouts
                   //                        only, 0 outside the image), else -1
    int stride;    // bytes per class (multiple of 256)
};

struct KParams {
    int W;         // model window side
    int B;         // target block side
    int off;       // (W - B) / 2
    int iters;     // nu_max
    double gamma;  // gamma_odc
    double ecoef;  // 2 gamma - gamma^2
    double tau;    // energy floor (0 = off)
    int dft_bf16;  // window DFT with split-BF16 MFMA products (FP32 plans)
    int shape;     // pixel-shape mask (0xE three-quarter, 0x1 quarter) or
                   // SHAPE_GENERAL: picks the kernel instantiation on the host
    DevConsts c;
    ClassLayout lay;
};

// One image as seen by the kernels.
struct KJob {
    const void *y;                 // sensor image, Ms x Ns
    void *out;                     // 2Ms x 2Ns
    const unsigned char *tables;   // class blocks
    const int *rowcls;             // [nbi] row key index
    const int *colcls;             // [nbj] column key index
    int16_t *sel;                  // [nwin][iters] or null
    int Ms, Ns, nbi, nbj, ncolk;
    int y64;                       // measurements are double (FP64 plans, and FP32 plans
                                   // made with LJSDE_INPUT_F64), else float
    long long win_begin;           // first global window index of this job
    const void *dense;             // dense C of the job's size set (batched dense form), else null
};

// Up to four windows of one job that share a class (persistent FP32 path).
struct WinGroup {
    int job;
    int count;
    int win[4];  // window index inside the job, row-major block order
};

// Launch wrappers (ljsde_kernels.hip, ljsde_mixed.hip). Return a hipError_t value.
int launch_plain_f64(const KParams &p, const KJob &job, int ws, void *stream);
int launch_plain_f32(const KParams &p, const KJob &job, int ws, void *stream);
// Zeroes the COUNTERS work counters of a batch (a fill kernel, so that the
// reset can sit in a captured graph).
constexpr int COUNTERS = 8;
int launch_reset_counter(unsigned int *counters, void *stream);
int launch_persistent_f32(const KParams &p, const KJob *d_jobs, int njobs, long long total_windows,
                          unsigned int *counter, int ws, int waves_per_block, int chunk,
                          int grid, void *stream);
int persistent_blocks_per_cu(int ws, int waves_per_block, int *blocks);
size_t lds_bytes_per_wave(int ws, bool fp64);
int launch_mixed_window(const KParams &p, const KJob &job, int ws, void *stream);
// Group ranges of the persistent FP32 launch: one per XCD of an MI355X.
// range_begin holds XCD_RANGES + 1 offsets into the group list.
constexpr int XCD_RANGES = COUNTERS;
// Launch variant of the persistent FP32 kernel (the autotuner's knobs).
struct MixedVariant {
    int nw = 4;         // windows (wavefronts) per workgroup: 1, 2 or 4
    int chunk = 1;      // groups taken per claim
    bool qreg = false;  // per-lane q/D and twiddles in registers instead of LDS
    bool vdft = false;  // window DFT as VALU passes instead of FP64 MFMA
};
int launch_mixed_persistent(const KParams &p, const KJob *d_jobs, const WinGroup *d_groups, const int *range_begin,
                            unsigned int *counters, int ws, const MixedVariant &v, int grid, void *stream);
int mixed_blocks_per_cu(int ws, const MixedVariant &v, int *blocks);
// Dense form (ljsde_dense.hip): bytes of the dense C of n classes, its build
// from the class tables, and the one-wavefront-per-window FP64 launch.
size_t dense_c_bytes(int ws, int n_classes);
int launch_dense_c_build(const KParams &p, const unsigned char *tables, int n_classes, int ws, void *out,
                         void *stream);
// order: window index per workgroup (-1: idle), order_len entries.
// f32io: float measurements and output (FP32 plans), else double.
int launch_dense(const KParams &p, const KJob &job, const void *C, const int *order, int order_len, int ws,
                 bool f32io, void *stream);

// Plain L-JSDE (ljsde_lplain.hip): up to LGROUP windows of one class per
// workgroup. `count` 0 marks an idle workgroup.
constexpr int LGROUP = 16;
struct LGroup {
    int cls;
    int count;
    int win[LGROUP];  // window index inside the job, row-major block order
};
// Bytes of the basis responses a of n classes ([cls][W^2/16][(W/2)^2][16] complex)
// and of their normalisers ([cls][2][W^2]: q/D, 1/D).
size_t lplain_a_bytes(int ws, int n_classes);
size_t lplain_aux_bytes(int ws, int n_classes);
// Builds a (eq. (10): a_m(f) = sum A_m(eta, gamma) Phi(eta, gamma, f)) and, from it, D
// of eq. (10) with q/D and 1/D for every class of a size set.
int launch_lplain_build(const KParams &p, const unsigned char *tables, int n_classes, int ws, void *a, void *aux,
                        void *stream);
// Batched dense form: `order` is int2 [n] = (job, window) per workgroup
// (job < 0: idle); every job carries its dense C in KJob::dense.
int launch_dense_batch(const KParams &p, const KJob *jobs, const void *order, int n, int ws, bool f32io,
                       void *stream);
// f32io: float output (FP32 plans; FP64 arithmetic), else double.
int launch_lplain(const KParams &p, const KJob &job, const void *a, const void *aux, const LGroup *groups,
                  int ngroups, int ws, bool f32io, void *stream);

// Allocation-free single-image launch of the persistent FP32 kernel. Its work
// memory (counters, group ranges, the job and the window groups) is a
// file-scope device array in ljsde_mixed.hip, one copy per GPU, of
// NOALLOC_BYTES; the work list holds at most NOALLOC_MAX_GROUPS groups.
constexpr int NOALLOC_MAX_GROUPS = 1 << 18;
constexpr size_t NOALLOC_OFF_RANGES = 256;   // int [XCD_RANGES + 1]
constexpr size_t NOALLOC_OFF_JOB = 512;      // KJob
constexpr size_t NOALLOC_OFF_GROUPS = 1024;  // WinGroup [NOALLOC_MAX_GROUPS]
constexpr size_t NOALLOC_BYTES = NOALLOC_OFF_GROUPS + (size_t)NOALLOC_MAX_GROUPS * sizeof(WinGroup);
// Device address of the array on device `dev` (the current device), looked
// up once per device. Returns a hipError_t value.
int noalloc_scratch(int dev, unsigned char **ptr);
// With `upload`, copies the host work list (which must outlive the copy) into
// the array; then one fill kernel writes the job, the ranges and zeroed
// counters, and the persistent kernel runs on them. Returns a hipError_t value.
int launch_mixed_noalloc(const KParams &p, const KJob &job, const WinGroup *host_groups, int ngroups,
                         const int *ranges, bool upload, int ws, const MixedVariant &v, int grid,
                         unsigned char *scr, void *stream);

}  // namespace ljsde
