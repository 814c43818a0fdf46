// Host runtime of the RL-JSDE library: plan registry, argument validation,
// enumeration of local measurement matrices ("classes"), FP64 precompute of
// the per-class tables, device upload and kernel launches.
//
// Sec. IV of the paper precomputes B, C and D once per local measurement
// matrix and reuses them for every window with the same one. For
// three-quarter sampling all of C factorises through four weighted-mask
// spectra S_o (one per opaque-quadrant orientation), so a class costs a few
// tens of KiB instead of the dense C of W^4 complex entries. General layouts
// (per-pixel quadrant weights) keep ten spectra S_qq' per class and run on
// the dense form, whose C is built on the device from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "../../include/ljsde.h"
#include "ljsde_internal.h"

namespace ljsde {
namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok() {
    g_last_error.clear();
    return LJSDE_OK;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? LJSDE_ENOMEM : LJSDE_EHIP, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                    \
    } while (0)

inline int pmod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// Pending simulated allocation failure (test hook, environment LJSDE_FAULT=alloc).
bool fault_alloc() {
    const char *f = getenv("LJSDE_FAULT");
    return f && strcmp(f, "alloc") == 0;
}

struct AxisKey {
    int phase, lo, hi;
    bool operator<(const AxisKey &o) const {
        return std::tie(phase, lo, hi) < std::tie(o.phase, o.lo, o.hi);
    }
};

// Tables of one image size for one plan.
struct SizeSet {
    int Ms = 0, Ns = 0, nbi = 0, nbj = 0;
    std::vector<AxisKey> rowkeys, colkeys;
    std::vector<int> rowcls, colcls;  // per block row / column
    int n_classes() const { return (int)(rowkeys.size() * colkeys.size()); }
    // host FP64 tables (built on demand)
    bool host_built = false;
    std::vector<unsigned char> blob;  // n_classes * layout.stride bytes
    std::vector<double> D;            // n_classes * W * W, normaliser of eq. (13)
    // device copies
    int device = -1;
    unsigned char *d_tables = nullptr;
    int *d_rowcls = nullptr;
    int *d_colcls = nullptr;
    void *d_dense = nullptr;  // dense C of every class (LJSDE_DENSE_C plans), built on first use
    int *d_order = nullptr;   // dense form: window of every workgroup (-1: none), see dense_order
    int order_len = 0;
    void *d_la = nullptr;      // plain L-JSDE: basis responses a of every class, built on first use
    void *d_laux = nullptr;    // plain L-JSDE: q/D and 1/D of every class
    LGroup *d_lgroups = nullptr;  // plain L-JSDE: window groups in launch order
    int n_lgroups = 0;
    // host work lists of the allocation-free entry point, per group width
    struct GroupList {
        std::vector<WinGroup> groups;
        int ranges[XCD_RANGES + 1];
    };
    std::map<int, GroupList> noalloc_lists;
};

struct Plan {
    std::vector<uint8_t> pattern;
    int pr = 0, pc = 0, W = 0, B = 0, Ws = 0, iters = 0;
    double rho = 0, gamma = 0, tau = 0;
    unsigned flags = 0;
    int shape = 0xE;                    // pixel-shape mask of quadrant offsets, or SHAPE_GENERAL
    std::vector<double> quad;           // general layouts: [pr][pc][4] quadrant weights per pixel
    ClassLayout lay{};
    std::vector<double> w, ew, dft, q, H;  // class-independent FP64 tables
    int device = -1;
    double *d_consts = nullptr;         // w | ew | dft | H | q
    std::map<std::pair<int, int>, std::unique_ptr<SizeSet>> sizes;
    bool fp64() const { return (flags & LJSDE_FP64) != 0; }
    bool general() const { return shape == SHAPE_GENERAL; }
    int n_spectra() const { return general() ? 10 : 4; }
};

std::mutex g_mu;
std::vector<std::unique_ptr<Plan>> g_plans;

ClassLayout make_layout(int W, int Ws, bool general) {
    ClassLayout L{};
    auto al = [](int x) { return (x + 255) & ~255; };
    int off = 0;
    L.offS = off;
    off = al(off + Ws * Ws * (general ? 10 : 4) * 2 * (int)sizeof(double));
    L.offQD64 = off;
    off = al(off + W * W * (int)sizeof(double));
    L.offInvD = off;
    off = al(off + W * W * (int)sizeof(double));
    L.offQD32 = off;
    off = al(off + W * W * (int)sizeof(float));
    L.offCodes = off;
    off = al(off + Ws * Ws);
    L.offA = -1;
    if (general) {
        L.offA = off;
        off = al(off + Ws * Ws * 4 * (int)sizeof(double));
    }
    L.stride = off;
    return L;
}

// Class-independent tables: spatial weights (eq. (8)), frequency weights
// q, and the twiddles of the W-point basis (Sec. III) and of the Ws-point
// sensor-grid DFT.
void build_constants(Plan &p) {
    const int W = p.W, Ws = p.Ws;
    p.w.resize(Ws * Ws);
    const double c = (W - 1) / 2.0;
    for (int i = 0; i < Ws; ++i)
        for (int j = 0; j < Ws; ++j) {
            const double di = 2 * i + 0.5 - c, dj = 2 * j + 0.5 - c;
            p.w[i * Ws + j] = std::pow(p.rho, std::sqrt(di * di + dj * dj));
        }
    p.ew.resize(2 * W);
    for (int k = 0; k < W; ++k) {
        const double a = 2.0 * M_PI * k / W;
        p.ew[2 * k] = std::cos(a);
        p.ew[2 * k + 1] = std::sin(a);
    }
    p.dft.resize(2 * Ws);
    for (int k = 0; k < Ws; ++k) {
        const double a = -2.0 * M_PI * k / Ws;
        p.dft[2 * k] = std::cos(a);
        p.dft[2 * k + 1] = std::sin(a);
    }
    // H_o(sigma, rho) = sum over the quadrants (a, b) that the pixel of code o
    // collects (q = 2a + b with bit q ^ o of the shape mask set) of
    // e^{i theta (a sigma + b rho)}; for three-quarter sampling, the box
    // response minus the opaque quadrant's term
    p.H.resize((size_t)W * W * 8);
    for (int sg = 0; sg < W; ++sg)
        for (int rh = 0; rh < W; ++rh)
            for (int o = 0; o < 4; ++o) {
                double hr = 0.0, hi = 0.0;
                for (int q = 0; q < 4; ++q) {
                    if (!((p.shape >> (q ^ o)) & 1)) continue;
                    const int ph = ((q >> 1) * sg + (q & 1) * rh) % W;
                    hr += p.ew[2 * ph];
                    hi += p.ew[2 * ph + 1];
                }
                p.H[((size_t)(sg * W + rh) * 4 + o) * 2] = hr;
                p.H[((size_t)(sg * W + rh) * 4 + o) * 2 + 1] = hi;
            }
    p.q.resize(W * W);
    const double qmax = std::sqrt(2.0) * W / 2.0;
    for (int s = 0; s < W; ++s)
        for (int r = 0; r < W; ++r) {
            if (p.flags & LJSDE_Q_ONES) {
                p.q[s * W + r] = 1.0;
                continue;
            }
            const double st = std::min(s, W - s), rt = std::min(r, W - r);
            const double x = 1.0 - std::sqrt(st * st + rt * rt) / qmax;
            p.q[s * W + r] = x * x;
        }
}

AxisKey axis_key(const Plan &p, int b, int Msens, int period) {
    const int s0 = (p.B * b - (p.W - p.B) / 2) / 2;  // window's first sensor row
    AxisKey k;
    k.lo = std::max(0, -s0);
    k.hi = std::max(0, s0 + p.Ws - Msens);
    k.phase = pmod(s0, period);
    return k;
}

void enumerate(const Plan &p, SizeSet &s) {
    s.nbi = 2 * s.Ms / p.B;
    s.nbj = 2 * s.Ns / p.B;
    std::map<AxisKey, int> rk, ck;
    s.rowcls.resize(s.nbi);
    s.colcls.resize(s.nbj);
    for (int b = 0; b < s.nbi; ++b) {
        AxisKey k = axis_key(p, b, s.Ms, p.pr);
        auto it = rk.find(k);
        if (it == rk.end()) {
            it = rk.emplace(k, (int)s.rowkeys.size()).first;
            s.rowkeys.push_back(k);
        }
        s.rowcls[b] = it->second;
    }
    for (int b = 0; b < s.nbj; ++b) {
        AxisKey k = axis_key(p, b, s.Ns, p.pc);
        auto it = ck.find(k);
        if (it == ck.end()) {
            it = ck.emplace(k, (int)s.colkeys.size()).first;
            s.colkeys.push_back(k);
        }
        s.colcls[b] = it->second;
    }
}

// A frequency whose D (eq. (13)) is at most D_REL times the class's largest
// D has no response in any measurement of the window (its exact D is 0; the
// computed one is rounding noise, eq. (16) is undefined): unobserved, metric 0.
constexpr double D_REL = 1e-13;

// q / D and 1 / D of one class, 0 at unobserved frequencies
void store_normaliser(const Plan &p, const double *D, unsigned char *dst) {
    double *qd = (double *)(dst + p.lay.offQD64);
    double *inv = (double *)(dst + p.lay.offInvD);
    float *qd32 = (float *)(dst + p.lay.offQD32);
    double dmax = 0.0;
    for (int f = 0; f < p.W * p.W; ++f) dmax = std::max(dmax, D[f]);
    for (int f = 0; f < p.W * p.W; ++f) {
        const bool pos = D[f] > 0 && D[f] > D_REL * dmax;
        qd[f] = pos ? p.q[f] / D[f] : 0.0;
        inv[f] = pos ? 1.0 / D[f] : 0.0;
        qd32[f] = (float)qd[f];
    }
}

// 2-D Ws-point DFT of a real tile v [Ws][Ws]:
// out[(k * Ws + l) * ostride + {0, 1}] = sum_{i, j} v(i, j) e^{-2 pi i (i k + j l) / Ws}, row pass first.
void dft2_real(const Plan &p, const double *v, double *out, int ostride) {
    const int Ws = p.Ws;
    std::vector<double> A((size_t)Ws * Ws * 2, 0.0);  // [i][l][re, im]
    for (int i = 0; i < Ws; ++i)
        for (int l = 0; l < Ws; ++l) {
            double re = 0, im = 0;
            for (int j = 0; j < Ws; ++j) {
                const int t = (j * l) % Ws;
                re += v[i * Ws + j] * p.dft[2 * t];
                im += v[i * Ws + j] * p.dft[2 * t + 1];
            }
            A[(i * Ws + l) * 2] = re;
            A[(i * Ws + l) * 2 + 1] = im;
        }
    for (int k = 0; k < Ws; ++k)
        for (int l = 0; l < Ws; ++l) {
            double re = 0, im = 0;
            for (int i = 0; i < Ws; ++i) {
                const int t = (i * k) % Ws;
                const double ar = A[(i * Ws + l) * 2], ai = A[(i * Ws + l) * 2 + 1];
                re += ar * p.dft[2 * t] - ai * p.dft[2 * t + 1];
                im += ar * p.dft[2 * t + 1] + ai * p.dft[2 * t];
            }
            out[(size_t)(k * Ws + l) * ostride] = re;
            out[(size_t)(k * Ws + l) * ostride + 1] = im;
        }
}

// Per-class FP64 tables of a general layout (Sec. II, eq. (1): pixel m weighs
// quadrant q = 2a + b of its footprint by A_m(q)). With
// a_m(f) = exp(i theta 2 (i' sigma + j' rho)) sum_q A_m(q) e_q(f) and
// e_q(f) = exp(i theta (a sigma + b rho)), C of eq. (14) is
// sum_{q, q'} conj(e_q(f)) e_q'(g) S_qq'(f - g) with the ten spectra
// S_qq' = DFT(w A_q A_q') (q <= q'), and D of eq. (13) is C(f, f).
void build_class_general(const Plan &p, const AxisKey &rk, const AxisKey &ck, unsigned char *dst, double *Dout) {
    const int W = p.W, Ws = p.Ws;
    std::vector<double> A((size_t)Ws * Ws * 4, 0.0);
    signed char *cd = (signed char *)(dst + p.lay.offCodes);
    for (int i = 0; i < Ws; ++i)
        for (int j = 0; j < Ws; ++j) {
            const bool valid = i >= rk.lo && i < Ws - rk.hi && j >= ck.lo && j < Ws - ck.hi;
            cd[i * Ws + j] = valid ? 0 : -1;
            if (!valid) continue;
            const double *src = &p.quad[((size_t)pmod(rk.phase + i, p.pr) * p.pc + pmod(ck.phase + j, p.pc)) * 4];
            for (int q = 0; q < 4; ++q) A[(i * Ws + j) * 4 + q] = src[q];
        }
    memcpy(dst + p.lay.offA, A.data(), A.size() * sizeof(double));
    double *S = (double *)(dst + p.lay.offS);
    std::vector<double> v((size_t)Ws * Ws);
    double mass[4][4];
    int idx = 0;
    for (int q = 0; q < 4; ++q)
        for (int r = q; r < 4; ++r, ++idx) {
            for (int m = 0; m < Ws * Ws; ++m) v[m] = p.w[m] * A[m * 4 + q] * A[m * 4 + r];
            dft2_real(p, v.data(), S + 2 * idx, 20);
            mass[q][r] = mass[r][q] = S[2 * idx];  // S_qq'(0, 0)
        }
    for (int sg = 0; sg < W; ++sg)
        for (int rh = 0; rh < W; ++rh) {
            double D = 0;
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 4; ++r) {
                    const int ph = pmod(((r >> 1) - (q >> 1)) * sg + ((r & 1) - (q & 1)) * rh, W);
                    D += mass[q][r] * p.ew[2 * ph];  // Re conj(e_q) e_r
                }
            Dout[sg * W + rh] = D;
        }
    store_normaliser(p, Dout, dst);
}

// Per-class FP64 tables. With a_m(sigma, rho) = exp(i theta (2i' sigma + 2j' rho)) H_o(sigma, rho)
// the diagonal of C (eq. (13)) is D = sum_o |H_o|^2 S_o(0, 0).
void build_class(const Plan &p, const SizeSet &s, int cls, unsigned char *dst, double *Dout) {
    const int W = p.W, Ws = p.Ws;
    const AxisKey &rk = s.rowkeys[cls / (int)s.colkeys.size()];
    const AxisKey &ck = s.colkeys[cls % (int)s.colkeys.size()];
    if (p.general()) {
        build_class_general(p, rk, ck, dst, Dout);
        return;
    }
    std::vector<int> code(Ws * Ws);
    for (int i = 0; i < Ws; ++i)
        for (int j = 0; j < Ws; ++j) {
            const bool valid = i >= rk.lo && i < Ws - rk.hi && j >= ck.lo && j < Ws - ck.hi;
            code[i * Ws + j] =
                valid ? p.pattern[pmod(rk.phase + i, p.pr) * p.pc + pmod(ck.phase + j, p.pc)] : -1;
        }
    // S_o(k, l) = sum_{i, j: code = o} w e^{-2 pi i (i k + j l) / Ws}, separable
    std::vector<double> A(4 * Ws * Ws * 2, 0.0);  // [o][i][l][re, im]
    for (int o = 0; o < 4; ++o)
        for (int i = 0; i < Ws; ++i)
            for (int l = 0; l < Ws; ++l) {
                double re = 0, im = 0;
                for (int j = 0; j < Ws; ++j) {
                    if (code[i * Ws + j] != o) continue;
                    const int t = (j * l) % Ws;
                    re += p.w[i * Ws + j] * p.dft[2 * t];
                    im += p.w[i * Ws + j] * p.dft[2 * t + 1];
                }
                A[((o * Ws + i) * Ws + l) * 2] = re;
                A[((o * Ws + i) * Ws + l) * 2 + 1] = im;
            }
    double *S = (double *)(dst + p.lay.offS);
    for (int k = 0; k < Ws; ++k)
        for (int l = 0; l < Ws; ++l)
            for (int o = 0; o < 4; ++o) {
                double re = 0, im = 0;
                for (int i = 0; i < Ws; ++i) {
                    const int t = (i * k) % Ws;
                    const double ar = A[((o * Ws + i) * Ws + l) * 2], ai = A[((o * Ws + i) * Ws + l) * 2 + 1];
                    re += ar * p.dft[2 * t] - ai * p.dft[2 * t + 1];
                    im += ar * p.dft[2 * t + 1] + ai * p.dft[2 * t];
                }
                S[((k * Ws + l) * 4 + o) * 2] = re;
                S[((k * Ws + l) * 4 + o) * 2 + 1] = im;
            }
    double mass[4];
    for (int o = 0; o < 4; ++o) mass[o] = S[o * 2];  // S_o(0, 0)
    for (int f = 0; f < W * W; ++f) {
        const double *H = &p.H[(size_t)f * 8];
        double D = 0;
        for (int o = 0; o < 4; ++o) D += (H[2 * o] * H[2 * o] + H[2 * o + 1] * H[2 * o + 1]) * mass[o];
        Dout[f] = D;
    }
    store_normaliser(p, Dout, dst);
    signed char *cd = (signed char *)(dst + p.lay.offCodes);
    for (int m = 0; m < Ws * Ws; ++m) cd[m] = (signed char)code[m];
}

void build_host_tables(const Plan &p, SizeSet &s) {
    if (s.host_built) return;
    const int n = s.n_classes();
    s.blob.assign((size_t)n * p.lay.stride, 0);
    s.D.assign((size_t)n * p.W * p.W, 0.0);
    for (int c = 0; c < n; ++c)
        build_class(p, s, c, s.blob.data() + (size_t)c * p.lay.stride, s.D.data() + (size_t)c * p.W * p.W);
    s.host_built = true;
}

int get_plan(int id, Plan **out) {
    if (id < 0 || id >= (int)g_plans.size() || !g_plans[id])
        return fail(LJSDE_EBADID, "unknown or released pattern id %d", id);
    *out = g_plans[id].get();
    return LJSDE_OK;
}

int check_size(const Plan &p, int Ms, int Ns) {
    if (Ms <= 0 || Ns <= 0) return fail(LJSDE_EINVAL, "sensor size %dx%d must be positive", Ms, Ns);
    if ((2 * Ms) % p.B || (2 * Ns) % p.B)
        return fail(LJSDE_EINVAL, "sensor size %dx%d: sides must be multiples of block/2 = %d", Ms, Ns,
                    p.B / 2);
    if ((long long)Ms * Ns > (1LL << 31) / 4)
        return fail(LJSDE_EUNSUPPORTED, "sensor size %dx%d too large", Ms, Ns);
    return LJSDE_OK;
}

int get_size(Plan &p, int Ms, int Ns, SizeSet **out) {
    int st = check_size(p, Ms, Ns);
    if (st) return st;
    auto key = std::make_pair(Ms, Ns);
    auto it = p.sizes.find(key);
    if (it == p.sizes.end()) {
        auto s = std::make_unique<SizeSet>();
        s->Ms = Ms;
        s->Ns = Ns;
        enumerate(p, *s);
        it = p.sizes.emplace(key, std::move(s)).first;
    }
    *out = it->second.get();
    return LJSDE_OK;
}

int current_device(int *dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(LJSDE_EHIP, "no HIP device available");
    HIP_TRY(hipGetDevice(dev));
    return LJSDE_OK;
}

int dev_alloc(void **p, size_t bytes) {
    if (fault_alloc()) return fail(LJSDE_ENOMEM, "simulated device allocation failure");
    HIP_TRY(hipMalloc(p, bytes));
    return LJSDE_OK;
}

int ensure_device(Plan &p, SizeSet &s) {
    int dev = 0;
    int st = current_device(&dev);
    if (st) return st;
    if (p.d_consts && p.device != dev)
        return fail(LJSDE_EUNSUPPORTED, "plan tables live on device %d, current device is %d", p.device,
                    dev);
    if (!p.d_consts) {
        std::vector<double> c;
        c.insert(c.end(), p.w.begin(), p.w.end());
        c.insert(c.end(), p.ew.begin(), p.ew.end());
        c.insert(c.end(), p.dft.begin(), p.dft.end());
        c.insert(c.end(), p.H.begin(), p.H.end());
        c.insert(c.end(), p.q.begin(), p.q.end());
        void *d = nullptr;
        st = dev_alloc(&d, c.size() * sizeof(double));
        if (st) return st;
        hipError_t e = hipMemcpy(d, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(LJSDE_EHIP, "upload of constants: %s", hipGetErrorString(e));
        }
        p.d_consts = (double *)d;
        p.device = dev;
    }
    if (!s.d_tables) {
        build_host_tables(p, s);
        void *dt = nullptr, *dr = nullptr, *dc = nullptr;
        st = dev_alloc(&dt, s.blob.size());
        if (st) return st;
        st = dev_alloc(&dr, s.rowcls.size() * sizeof(int));
        if (st) {
            (void)hipFree(dt);
            return st;
        }
        st = dev_alloc(&dc, s.colcls.size() * sizeof(int));
        if (st) {
            (void)hipFree(dt);
            (void)hipFree(dr);
            return st;
        }
        hipError_t e = hipMemcpy(dt, s.blob.data(), s.blob.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dr, s.rowcls.data(), s.rowcls.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dc, s.colcls.data(), s.colcls.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dt);
            (void)hipFree(dr);
            (void)hipFree(dc);
            return fail(LJSDE_EHIP, "upload of class tables: %s", hipGetErrorString(e));
        }
        s.d_tables = (unsigned char *)dt;
        s.d_rowcls = (int *)dr;
        s.d_colcls = (int *)dc;
        s.device = dev;
    }
    return LJSDE_OK;
}

KParams make_params(const Plan &p) {
    KParams k{};
    k.W = p.W;
    k.B = p.B;
    k.off = (p.W - p.B) / 2;
    k.iters = p.iters;
    k.gamma = p.gamma;
    k.ecoef = 2 * p.gamma - p.gamma * p.gamma;
    k.tau = p.tau;
    k.dft_bf16 = (p.flags & LJSDE_DFT_SPLITBF16) != 0 ? 1 : 0;
    k.shape = p.shape;
    k.c.w = p.d_consts;
    k.c.ew = p.d_consts + p.w.size();
    k.c.dft = p.d_consts + p.w.size() + p.ew.size();
    k.c.H = p.d_consts + p.w.size() + p.ew.size() + p.dft.size();
    k.c.q = k.c.H + p.H.size();
    k.lay = p.lay;
    return k;
}

KJob make_job(const Plan &p, const SizeSet &s, const void *y, void *out, int16_t *sel, long long win_begin) {
    KJob j{};
    j.y = y;
    j.y64 = (p.flags & (LJSDE_FP64 | LJSDE_INPUT_F64)) != 0 ? 1 : 0;
    j.out = out;
    j.tables = s.d_tables;
    j.rowcls = s.d_rowcls;
    j.colcls = s.d_colcls;
    j.sel = sel;
    j.Ms = s.Ms;
    j.Ns = s.Ns;
    j.nbi = s.nbi;
    j.nbj = s.nbj;
    j.ncolk = (int)s.colkeys.size();
    j.win_begin = win_begin;
    return j;
}

// ---------------------------------------------------------------------------
// Persistent batched launches
// ---------------------------------------------------------------------------

// Launch variant of a batch: windows per workgroup (same-class groups for
// the FP64-state path; independent windows for the FP32-state path) and, for
// the latter, windows per work grab.
struct TuneChoice {
    int waves_per_block = 4;
    int chunk = 2;         // FP32-state path: windows per grab; FP64-state path: groups per claim
    int fewer_blocks = 0;  // resident workgroups per CU below the occupancy maximum
    int qreg = 0;          // FP64-state path: per-lane q/D and twiddles held in registers
    int vdft = 0;          // FP64-state path: window DFT as VALU passes instead of FP64 MFMA
};

TuneChoice default_choice(bool state_fp32) { return state_fp32 ? TuneChoice{1, 2} : TuneChoice{4, 1, 0}; }

MixedVariant mixed_variant(const TuneChoice &c) {
    MixedVariant v;
    v.nw = c.waves_per_block;
    v.chunk = c.chunk;
    v.qreg = c.qreg != 0;
    v.vdft = c.vdft != 0;
    return v;
}

struct BatchState {
    bool state_fp32 = false;            // all-FP32 variant (LJSDE_STATE_FP32)
    std::vector<KJob> host_jobs;
    std::vector<const SizeSet *> sizes;  // host class maps of the jobs (owned by their plans)
    std::string tune_key;
    KJob *d_jobs = nullptr;
    WinGroup *d_groups = nullptr;
    int *d_ranges = nullptr;            // XCD_RANGES + 1 offsets into d_groups
    int ngroups = 0;
    int groups_nw = 0;                  // group width the device list was built for
    unsigned int *d_counter = nullptr;  // COUNTERS work counters
    long long total = 0;
    KParams params{};
    int ws = 16;
    int device = -1;
    TuneChoice choice;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchState() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_jobs) (void)hipFree(d_jobs);
        if (d_groups) (void)hipFree(d_groups);
        if (d_ranges) (void)hipFree(d_ranges);
        if (d_counter) (void)hipFree(d_counter);
    }
};

std::map<std::string, std::unique_ptr<BatchState>> g_batches;

// Batched dense form: the job table and the launch order, (job, window) per
// workgroup, kept per batch shape and stream like the FP32 batch states.
struct DenseBatch {
    std::vector<KJob> host_jobs;
    KJob *d_jobs = nullptr;
    int *d_order = nullptr;  // int2 [n_order]
    int n_order = 0;
    KParams params{};
    int ws = 16;
    bool f32io = false;
    ~DenseBatch() {
        if (d_jobs) (void)hipFree(d_jobs);
        if (d_order) (void)hipFree(d_order);
    }
};
std::map<std::string, std::unique_ptr<DenseBatch>> g_dense_batches;
std::map<std::string, TuneChoice> g_tuned;
hipStream_t g_capture_stream = nullptr;

std::string tune_key(const Plan &p, bool state_fp32, long long total_windows, int n_classes) {
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    int bucket = 0;
    while ((1 << bucket) < n_classes) ++bucket;
    int wb = 0;
    while ((1LL << wb) < total_windows) ++wb;
    std::ostringstream os;
    os << prop.gcnArchName << "/W" << p.W << "/B" << p.B << "/it" << p.iters
       << (state_fp32 ? "/fp32" : "/fp32s64") << "/s" << p.shape << "/c" << bucket << "/n" << wb;
    return os.str();
}

void load_tune_cache() {
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char *path = getenv("LJSDE_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    std::string line;
    // one entry per line: "key" : [waves_per_block, chunk, fewer_blocks, qreg, vdft]
    // (entries of three numbers: qreg = vdft = 0)
    while (std::getline(f, line)) {
        size_t a = line.find('"');
        if (a == std::string::npos) continue;
        size_t b = line.find('"', a + 1);
        if (b == std::string::npos) continue;
        size_t l = line.find('[', b);
        if (l == std::string::npos || line.find(']', l) == std::string::npos) continue;
        TuneChoice c;
        const int n = sscanf(line.c_str() + l + 1, "%d , %d , %d , %d , %d", &c.waves_per_block, &c.chunk,
                             &c.fewer_blocks, &c.qreg, &c.vdft);
        if ((n == 3 || n == 5) &&
            (c.waves_per_block == 1 || c.waves_per_block == 2 || c.waves_per_block == 4) && c.chunk >= 1 &&
            c.chunk <= 64 && c.fewer_blocks >= 0 && c.fewer_blocks < 8 && (c.qreg == 0 || c.qreg == 1) &&
            (c.vdft == 0 || c.vdft == 1))
            g_tuned[line.substr(a + 1, b - a - 1)] = c;
    }
}

// Written to a temporary file beside the cache and renamed over it, so that
// processes sharing the cache never read a partly written file.
void save_tune_cache() {
    const char *path = getenv("LJSDE_TUNE_CACHE");
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t i = 0;
        for (auto &kv : g_tuned) {
            f << "  \"" << kv.first << "\" : [" << kv.second.waves_per_block << ", " << kv.second.chunk << ", "
              << kv.second.fewer_blocks << ", " << kv.second.qreg << ", " << kv.second.vdft << "]"
              << (++i < g_tuned.size() ? "," : "") << "\n";
        }
        f << "}\n";
        if (!f) {
            f.close();
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

// Test hook: LJSDE_VARIANT="nw,chunk,fewer,qreg,vdft" forces the launch
// variant of batch states created afterwards (ignored when malformed).
void forced_variant(TuneChoice *c) {
    const char *v = getenv("LJSDE_VARIANT");
    if (!v) return;
    TuneChoice f;
    if (sscanf(v, "%d,%d,%d,%d,%d", &f.waves_per_block, &f.chunk, &f.fewer_blocks, &f.qreg, &f.vdft) == 5 &&
        (f.waves_per_block == 1 || f.waves_per_block == 2 || f.waves_per_block == 4) && f.chunk >= 1 &&
        f.chunk <= 64 && f.fewer_blocks >= 0 && f.fewer_blocks < 8 && (f.qreg == 0 || f.qreg == 1) &&
        (f.vdft == 0 || f.vdft == 1))
        *c = f;
}

int grid_for_shape(int ws, bool state_fp32, const TuneChoice &c, int *grid) {
    int dev = 0, ncu = 0, blocks = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int e = state_fp32 ? persistent_blocks_per_cu(ws, c.waves_per_block, &blocks)
                             : mixed_blocks_per_cu(ws, mixed_variant(c), &blocks);
    if (e != 0 || blocks <= 0) return fail(LJSDE_EHIP, "occupancy query failed (%d)", e);
    // a grid below full occupancy can finish a batch in whole rounds
    *grid = ncu * std::max(1, blocks - c.fewer_blocks);
    return LJSDE_OK;
}

int grid_for(const BatchState &b, const TuneChoice &c, int *grid) { return grid_for_shape(b.ws, b.state_fp32, c, grid); }

// Work list of the persistent FP32 launch: groups of up to nw windows of one
// class (they share the class tables staged in LDS). Interior windows (no
// clip on either axis) are grouped inside spatial tiles of the block grid,
// at least twice the class period on each axis (the number of row / column
// keys bounds that period), so a group is four nearby windows, and the tiles
// are listed in row-major order. Windows clipped by the image border follow,
// listed class by class: a border class runs along a whole image edge, so
// inside the tiles its tables would be fetched by every XCD whose range
// crosses that edge. The list is cut into XCD_RANGES contiguous ranges of
// equal length.
void make_group_list(const std::vector<const SizeSet *> &sizes, int nw, std::vector<WinGroup> &groups,
                     int ranges[XCD_RANGES + 1]) {
    groups.clear();
    auto emit = [&](int job, const std::vector<int> &ws) {
        for (size_t k = 0; k < ws.size(); k += nw) {
            WinGroup g{};
            g.job = job;
            g.count = (int)std::min<size_t>(nw, ws.size() - k);
            for (int w = 0; w < 4; ++w) g.win[w] = ws[k + std::min(w, g.count - 1)];
            groups.push_back(g);
        }
    };
    for (size_t ji = 0; ji < sizes.size(); ++ji) {
        const SizeSet &s = *sizes[ji];
        const int nck = (int)s.colkeys.size();
        auto interior = [&](const AxisKey &k) { return k.lo == 0 && k.hi == 0; };
        const int tr = std::min(s.nbi, std::max(16, 2 * (int)s.rowkeys.size()));
        const int tc = std::min(s.nbj, std::max(16, 2 * (int)s.colkeys.size()));
        std::vector<std::vector<int>> by_class(s.n_classes());
        std::vector<int> used;  // classes met in the current tile, in first-seen order
        for (int r0 = 0; r0 < s.nbi; r0 += tr)
            for (int c0 = 0; c0 < s.nbj; c0 += tc) {
                for (int bi = r0; bi < std::min(s.nbi, r0 + tr); ++bi)
                    for (int bj = c0; bj < std::min(s.nbj, c0 + tc); ++bj) {
                        if (!interior(s.rowkeys[s.rowcls[bi]]) || !interior(s.colkeys[s.colcls[bj]])) continue;
                        const int cls = s.rowcls[bi] * nck + s.colcls[bj];
                        if (by_class[cls].empty()) used.push_back(cls);
                        by_class[cls].push_back(bi * s.nbj + bj);
                    }
                for (int cls : used) {
                    emit((int)ji, by_class[cls]);
                    by_class[cls].clear();
                }
                used.clear();
            }
        // border windows, class by class (row-major inside a class)
        for (int bi = 0; bi < s.nbi; ++bi)
            for (int bj = 0; bj < s.nbj; ++bj)
                if (!interior(s.rowkeys[s.rowcls[bi]]) || !interior(s.colkeys[s.colcls[bj]]))
                    by_class[s.rowcls[bi] * nck + s.colcls[bj]].push_back(bi * s.nbj + bj);
        for (int cls = 0; cls < s.n_classes(); ++cls) {
            if (!by_class[cls].empty()) emit((int)ji, by_class[cls]);
            by_class[cls].clear();
        }
    }
    for (int r = 0; r <= XCD_RANGES; ++r) ranges[r] = (int)((long long)groups.size() * r / XCD_RANGES);
}

int build_groups(BatchState &b, int nw) {
    if (b.groups_nw == nw && b.d_groups) return LJSDE_OK;
    std::vector<WinGroup> groups;
    int ranges[XCD_RANGES + 1];
    make_group_list(b.sizes, nw, groups, ranges);
    if (b.d_groups) {
        (void)hipFree(b.d_groups);
        b.d_groups = nullptr;
    }
    int st = dev_alloc((void **)&b.d_groups, sizeof(WinGroup) * std::max<size_t>(groups.size(), 1));
    if (st) return st;
    if (!b.d_ranges) {
        st = dev_alloc((void **)&b.d_ranges, sizeof(ranges));
        if (st) return st;
    }
    HIP_TRY(hipMemcpy(b.d_groups, groups.data(), sizeof(WinGroup) * groups.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b.d_ranges, ranges, sizeof(ranges), hipMemcpyHostToDevice));
    b.ngroups = (int)groups.size();
    b.groups_nw = nw;
    return LJSDE_OK;
}

// A caller's buffer must be device (or managed) memory of the current device:
// a kernel handed a host pointer would fault. job < 0 names no batch job.
static int check_device_buffer(const void *ptr, const char *what, int job) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipPointerAttribute_t a{};
    const hipError_t e = hipPointerGetAttributes(&a, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // the query's error is not the caller's
        if (job >= 0) return fail(LJSDE_EINVAL, "job %d: %s is not device memory", job, what);
        return fail(LJSDE_EINVAL, "%s is not device memory", what);
    }
    const bool device = a.type == hipMemoryTypeDevice && a.device == dev;
    const bool managed = a.type == hipMemoryTypeManaged || a.isManaged;
    if (!device && !managed) {
        if (job >= 0)
            return fail(LJSDE_EINVAL, "job %d: %s is not memory of device %d (memory type %d, device %d)", job,
                        what, dev, (int)a.type, a.device);
        return fail(LJSDE_EINVAL, "%s is not memory of device %d (memory type %d, device %d)", what, dev,
                    (int)a.type, a.device);
    }
    return LJSDE_OK;
}

// Builds (or finds) the batch state for this shape, refreshes the device job
// table if the buffers changed, and returns it.
int prepare_batch(const ljsde_job *jobs, int n, void *stream, BatchState **out) {
    if (!jobs || n <= 0) return fail(LJSDE_EINVAL, "empty batch");
    Plan *p0 = nullptr;
    int st = get_plan(jobs[0].pattern_id, &p0);
    if (st) return st;
    const bool sf32 = (p0->flags & LJSDE_STATE_FP32) != 0;
    std::ostringstream key;
    for (int i = 0; i < n; ++i) {
        Plan *p = nullptr;
        st = get_plan(jobs[i].pattern_id, &p);
        if (st) return st;
        if (p->fp64()) return fail(LJSDE_EUNSUPPORTED, "job %d: batched launches need FP32 plans", i);
        if (p->flags & (LJSDE_DENSE_C | LJSDE_PLAIN_L))
            return fail(LJSDE_EUNSUPPORTED, "job %d: batched launches need FP32 plans of the factorised form", i);
        // one launch reads the class-independent tables (spatial weights of
        // eq. (8), pixel responses) of the first plan
        if (p->W != p0->W || p->B != p0->B || p->iters != p0->iters || p->gamma != p0->gamma ||
            p->rho != p0->rho || p->tau != p0->tau || ((p->flags & LJSDE_STATE_FP32) != 0) != sf32 ||
            p->shape != p0->shape || ((p->flags ^ p0->flags) & LJSDE_DFT_SPLITBF16))
            return fail(LJSDE_EINVAL, "job %d: all plans of a batch need equal window, block, iters, rho, "
                                      "gamma, energy floor, state precision, DFT mode and pixel shape", i);
        if (!jobs[i].measurements || !jobs[i].out)
            return fail(LJSDE_EINVAL, "job %d: null device pointer", i);
        st = check_size(*p, jobs[i].sensor_rows, jobs[i].sensor_cols);
        if (st) return st;
        key << jobs[i].pattern_id << ':' << jobs[i].sensor_rows << 'x' << jobs[i].sensor_cols << ';';
    }
    int dev = 0;
    st = current_device(&dev);
    if (st) return st;
    // one state per stream: launches on different streams may overlap, and
    // each needs its own work counters and job table
    key << "@" << dev << "/s" << (uintptr_t)stream;
    auto &slot = g_batches[key.str()];
    if (!slot) {
        auto b = std::make_unique<BatchState>();
        b->state_fp32 = sf32;
        long long total = 0;
        int n_classes = 0;
        for (int i = 0; i < n; ++i) {
            Plan *p = nullptr;
            get_plan(jobs[i].pattern_id, &p);
            SizeSet *s = nullptr;
            st = get_size(*p, jobs[i].sensor_rows, jobs[i].sensor_cols, &s);
            if (st) return st;
            st = ensure_device(*p, *s);
            if (st) return st;
            b->host_jobs.push_back(make_job(*p, *s, nullptr, nullptr, nullptr, total));
            b->sizes.push_back(s);
            total += (long long)s->nbi * s->nbj;
            n_classes = std::max(n_classes, s->n_classes());
        }
        if (total >= (1LL << 31)) return fail(LJSDE_EUNSUPPORTED, "batch has too many windows");
        b->total = total;
        b->params = make_params(*p0);
        b->ws = p0->Ws;
        b->device = dev;
        b->tune_key = tune_key(*p0, sf32, total, n_classes);
        b->choice = default_choice(sf32);
        st = dev_alloc((void **)&b->d_jobs, sizeof(KJob) * n);
        if (st) return st;
        st = dev_alloc((void **)&b->d_counter, sizeof(unsigned int) * COUNTERS);
        if (st) return st;
        load_tune_cache();
        auto t = g_tuned.find(b->tune_key);
        if (t != g_tuned.end()) b->choice = t->second;
        forced_variant(&b->choice);
        st = grid_for(*b, b->choice, &b->grid);
        if (st) return st;
        if (!sf32) {
            st = build_groups(*b, b->choice.waves_per_block);
            if (st) return st;
        }
        slot = std::move(b);
    }
    BatchState *b = slot.get();
    bool changed = false;
    for (int i = 0; i < n; ++i) {
        KJob &j = b->host_jobs[i];
        if (j.y != jobs[i].measurements || j.out != jobs[i].out) {
            j.y = jobs[i].measurements;
            j.out = jobs[i].out;
            changed = true;
        }
    }
    if (changed) {
        for (int i = 0; i < n; ++i) {
            if ((st = check_device_buffer(jobs[i].measurements, "measurements", i)) ||
                (st = check_device_buffer(jobs[i].out, "out", i))) {
                for (int k = 0; k < n; ++k) b->host_jobs[k].y = b->host_jobs[k].out = nullptr;  // re-check next call
                return st;
            }
        }
        if (stream) HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        HIP_TRY(hipMemcpy(b->d_jobs, b->host_jobs.data(), sizeof(KJob) * n, hipMemcpyHostToDevice));
    }
    *out = b;
    return LJSDE_OK;
}

int launch_batch_eager(BatchState &b, const TuneChoice &c, int grid, void *stream) {
    int e = launch_reset_counter(b.d_counter, stream);
    if (e) return fail(LJSDE_EHIP, "reset launch: %s", hipGetErrorString((hipError_t)e));
    if (b.state_fp32)
        e = launch_persistent_f32(b.params, b.d_jobs, (int)b.host_jobs.size(), b.total, b.d_counter, b.ws,
                                  c.waves_per_block, c.chunk, grid, stream);
    else
        e = launch_mixed_persistent(b.params, b.d_jobs, b.d_groups, b.d_ranges, b.d_counter, b.ws,
                                    mixed_variant(c), grid, stream);
    if (e) return fail(LJSDE_EHIP, "persistent launch: %s", hipGetErrorString((hipError_t)e));
    return LJSDE_OK;
}

void drop_graph(BatchState &b) {
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
}

// Captures the batch's launch for its current choice; the work list is
// (re)built for that choice first, so the graph never refers to a list that
// the autotuner replaced.
int capture_graph(BatchState &b) {
    if (!g_capture_stream) HIP_TRY(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    drop_graph(b);
    int st = grid_for(b, b.choice, &b.grid);
    if (st) return st;
    if (!b.state_fp32) {
        st = build_groups(b, b.choice.waves_per_block);
        if (st) return st;
    }
    HIP_TRY(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    st = launch_batch_eager(b, b.choice, b.grid, g_capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(g_capture_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(LJSDE_EHIP, "graph capture: %s", hipGetErrorString(e));
    b.graph = g;
    HIP_TRY(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    return LJSDE_OK;
}

// Frees the batch states whose jobs use this plan (their keys list the
// pattern ids as "id:RxC;"), after the work in flight has completed.
template <typename M>
void drop_keyed(M &states, const std::string &pref, bool &synced) {
    for (auto it = states.begin(); it != states.end();) {
        const std::string &k = it->first;
        const bool uses = k.compare(0, pref.size(), pref) == 0 || k.find(";" + pref) != std::string::npos;
        if (!uses) {
            ++it;
            continue;
        }
        if (!synced) {
            (void)hipDeviceSynchronize();
            synced = true;
        }
        it = states.erase(it);
    }
}

void drop_batches_of(int pattern_id) {
    const std::string pref = std::to_string(pattern_id) + ":";
    bool synced = false;
    drop_keyed(g_batches, pref, synced);
    drop_keyed(g_dense_batches, pref, synced);
}

int run_batch(const ljsde_job *jobs, int n, void *stream) {
    BatchState *b = nullptr;
    int st = prepare_batch(jobs, n, stream, &b);
    if (st) return st;
    if (!b->exec) {
        st = capture_graph(*b);
        if (st) return st;
    }
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return ok();
}

}  // namespace
}  // namespace ljsde

using namespace ljsde;

extern "C" {

int ljsde_version(void) { return 10300; }  // 1.3: LJSDE_PLAIN_L, ljsde_reconstruct_noalloc (1.2: LJSDE_INPUT_F64; 1.1: ljsde_plan_weights, every pixel-shape mask)

int ljsde_plan_info(int pattern_id, int *window, int *block, int *iters, unsigned *flags) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    if (window) *window = p->W;
    if (block) *block = p->B;
    if (iters) *iters = p->iters;
    if (flags) *flags = p->flags;
    return ok();
}

const char *ljsde_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Checks shared by both plan constructors: pattern size, window geometry,
// iteration count, rho and gamma.
int check_plan_args(int pat_rows, int pat_cols, int window, int block, int iters, double rho, double gamma) {
    if (pat_rows <= 0 || pat_cols <= 0)
        return fail(LJSDE_EINVAL, "pattern size %dx%d must be positive", pat_rows, pat_cols);
    if ((long long)pat_rows * pat_cols > (1LL << 28)) return fail(LJSDE_EINVAL, "pattern too large");
    if (window <= 0 || block <= 0 || window % 2 || block % 2 || block > window || (window - block) % 4)
        return fail(LJSDE_EINVAL,
                    "window %d / block %d: need even sizes, block <= window, (window - block) %% 4 == 0",
                    window, block);
    if (iters < 1) return fail(LJSDE_EINVAL, "iters %d must be >= 1", iters);
    if (!(rho > 0.0 && rho <= 1.0)) return fail(LJSDE_EINVAL, "rho %g must be in (0, 1]", rho);
    if (!(gamma > 0.0 && gamma < 2.0)) return fail(LJSDE_EINVAL, "gamma %g must be in (0, 2)", gamma);
    return LJSDE_OK;
}

int register_plan(std::unique_ptr<Plan> p) {
    p->Ws = p->W / 2;
    p->lay = make_layout(p->W, p->Ws, p->general());
    build_constants(*p);
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.push_back(std::move(p));
    ok();
    return (int)g_plans.size() - 1;
}

}  // namespace

extern "C" {

int ljsde_plan(const uint8_t *pattern, int pat_rows, int pat_cols, int window, int block, int iters,
               double rho, double gamma, unsigned flags) {
    if (!pattern) return fail(LJSDE_EINVAL, "pattern is null");
    int st = check_plan_args(pat_rows, pat_cols, window, block, iters, rho, gamma);
    if (st) return st;
    for (long long i = 0; i < (long long)pat_rows * pat_cols; ++i)
        if (pattern[i] > 3) return fail(LJSDE_EINVAL, "pattern code %d at %lld not in 0..3", pattern[i], i);
    const unsigned known = LJSDE_FP64 | LJSDE_FP32 | LJSDE_DFT_SPLITBF16 | LJSDE_Q_ONES | LJSDE_STATE_FP32 |
                           LJSDE_DENSE_C | LJSDE_INPUT_F64 | LJSDE_SHAPE(15) | LJSDE_PLAIN_L;
    if (flags & ~known) return fail(LJSDE_EINVAL, "unknown flags 0x%x", flags & ~known);
    if (((flags & LJSDE_FP64) != 0) == ((flags & LJSDE_FP32) != 0))
        return fail(LJSDE_EINVAL, "exactly one of LJSDE_FP64 / LJSDE_FP32 is required");
    if ((flags & LJSDE_PLAIN_L) && (flags & (LJSDE_DENSE_C | LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)))
        return fail(LJSDE_EINVAL,
                    "LJSDE_PLAIN_L excludes LJSDE_DENSE_C, LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32");
    if ((flags & (LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)) && (flags & LJSDE_FP64))
        return fail(LJSDE_EINVAL, "LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32 apply to FP32 plans only");
    if ((flags & LJSDE_DENSE_C) && (flags & (LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)))
        return fail(LJSDE_EINVAL, "LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32 do not apply to the dense form");
    if (!(window == 32 || window == 16))
        return fail(LJSDE_EUNSUPPORTED, "no kernel for window %d (have 16, 32)", window);
    if ((flags & LJSDE_DFT_SPLITBF16) && window != 32)
        return fail(LJSDE_EUNSUPPORTED, "LJSDE_DFT_SPLITBF16 needs window 32");
    if (!(block == 4 || block == 8))
        return fail(LJSDE_EUNSUPPORTED, "no kernel for block %d (have 4, 8)", block);
    if (iters > 32767) return fail(LJSDE_EUNSUPPORTED, "iters %d above 32767", iters);
    int mask = (int)((flags >> 8) & 15u);
    if (mask == 0) mask = 0xE;
    const int bits = __builtin_popcount(mask);
    auto p = std::make_unique<Plan>();
    const size_t n = (size_t)pat_rows * pat_cols;
    p->pattern.assign(pattern, pattern + n);
    if (bits == 3 || bits == 1) {
        // Three collected quadrants: the pixel of code o misses o ^ d for the
        // one offset d outside the mask, i.e. three-quarter sampling with the
        // opaque quadrant o ^ d. One collected quadrant o ^ d: quarter
        // sampling with the transparent quadrant o ^ d. Relabel the codes.
        const int d = __builtin_ctz(bits == 3 ? (~mask & 15) : mask);
        for (auto &c : p->pattern) c = (uint8_t)(c ^ d);
        p->shape = bits == 3 ? 0xE : 0x1;
        if (p->shape == 0x1 && (flags & (LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)))
            return fail(LJSDE_EUNSUPPORTED,
                        "LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32 exist for three-quarter sampling only");
        p->flags = flags;
    } else {
        // Two or four collected quadrants (half, diagonal and full pixels):
        // their 0/1 quadrant weights through the general-layout dense form.
        if (!(flags & (LJSDE_DENSE_C | LJSDE_PLAIN_L)))
            return fail(LJSDE_EUNSUPPORTED,
                        "pixel shape mask 0x%x runs on the dense form (LJSDE_DENSE_C) or plain L-JSDE "
                        "(LJSDE_PLAIN_L) only", mask);
        p->quad.resize(n * 4);
        for (size_t i = 0; i < n; ++i)
            for (int q = 0; q < 4; ++q) p->quad[i * 4 + q] = (double)((mask >> (q ^ pattern[i])) & 1);
        p->shape = SHAPE_GENERAL;
        p->flags = flags | LJSDE_WEIGHTS;
    }
    p->pr = pat_rows;
    p->pc = pat_cols;
    p->W = window;
    p->B = block;
    p->iters = iters;
    p->rho = rho;
    p->gamma = gamma;
    return register_plan(std::move(p));
}

int ljsde_plan_weights(const double *weights, int pat_rows, int pat_cols, int window, int block, int iters,
                       double rho, double gamma, unsigned flags) {
    if (!weights) return fail(LJSDE_EINVAL, "weights is null");
    int st = check_plan_args(pat_rows, pat_cols, window, block, iters, rho, gamma);
    if (st) return st;
    const long long n = (long long)pat_rows * pat_cols * 4;
    for (long long i = 0; i < n; ++i)
        if (!std::isfinite(weights[i])) return fail(LJSDE_EINVAL, "weight %lld is not finite", i);
    const unsigned known = LJSDE_FP64 | LJSDE_FP32 | LJSDE_DFT_SPLITBF16 | LJSDE_Q_ONES | LJSDE_STATE_FP32 |
                           LJSDE_DENSE_C | LJSDE_INPUT_F64 | LJSDE_SHAPE(15) | LJSDE_WEIGHTS | LJSDE_PLAIN_L;
    if (flags & ~known) return fail(LJSDE_EINVAL, "unknown flags 0x%x", flags & ~known);
    if (flags & LJSDE_SHAPE(15)) return fail(LJSDE_EINVAL, "a pixel shape does not apply to a weights plan");
    if (((flags & LJSDE_FP64) != 0) == ((flags & LJSDE_FP32) != 0))
        return fail(LJSDE_EINVAL, "exactly one of LJSDE_FP64 / LJSDE_FP32 is required");
    if ((flags & (LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)) && (flags & LJSDE_FP64))
        return fail(LJSDE_EINVAL, "LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32 apply to FP32 plans only");
    if ((flags & LJSDE_DENSE_C) && (flags & (LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)))
        return fail(LJSDE_EINVAL, "LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32 do not apply to the dense form");
    if (!(window == 32 || window == 16))
        return fail(LJSDE_EUNSUPPORTED, "no kernel for window %d (have 16, 32)", window);
    if (!(block == 4 || block == 8))
        return fail(LJSDE_EUNSUPPORTED, "no kernel for block %d (have 4, 8)", block);
    if (iters > 32767) return fail(LJSDE_EUNSUPPORTED, "iters %d above 32767", iters);
    if ((flags & LJSDE_PLAIN_L) && (flags & (LJSDE_DENSE_C | LJSDE_DFT_SPLITBF16 | LJSDE_STATE_FP32)))
        return fail(LJSDE_EINVAL,
                    "LJSDE_PLAIN_L excludes LJSDE_DENSE_C, LJSDE_DFT_SPLITBF16 and LJSDE_STATE_FP32");
    if (!(flags & (LJSDE_DENSE_C | LJSDE_PLAIN_L)))
        return fail(LJSDE_EUNSUPPORTED,
                    "general layouts run on the dense form (LJSDE_DENSE_C) or plain L-JSDE (LJSDE_PLAIN_L) only");
    auto p = std::make_unique<Plan>();
    p->quad.assign(weights, weights + n);
    p->pattern.assign((size_t)pat_rows * pat_cols, 0);
    p->pr = pat_rows;
    p->pc = pat_cols;
    p->W = window;
    p->B = block;
    p->iters = iters;
    p->rho = rho;
    p->gamma = gamma;
    p->flags = flags | LJSDE_WEIGHTS;
    p->shape = SHAPE_GENERAL;
    return register_plan(std::move(p));
}

int ljsde_set_energy_floor(int pattern_id, double tau) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    if (!(tau >= 0.0 && tau < 1.0)) return fail(LJSDE_EINVAL, "tau %g must be in [0, 1)", tau);
    if (tau != p->tau) {
        p->tau = tau;
        // batch states hold the kernel parameters (and their graphs a copy of
        // them) from their creation: drop those of this plan, so that the next
        // batched call rebuilds them with the new floor
        drop_batches_of(pattern_id);
    }
    return ok();
}

// Launch order of the dense form: windows sorted by class (row-major inside a
// class) and cut into XCD_RANGES contiguous chunks of equal length; workgroup
// b runs entry b / XCD_RANGES of chunk b % XCD_RANGES. Workgroups are dealt
// to the XCDs round-robin, so each XCD works through a few classes at a time
// and their hot columns of C stay in its L2.
static std::vector<int> dense_order(const SizeSet &s) {
    const int n = s.nbi * s.nbj, nck = (int)s.colkeys.size();
    std::vector<int> win(n);
    for (int i = 0; i < n; ++i) win[i] = i;
    std::stable_sort(win.begin(), win.end(), [&](int a, int b) {
        return s.rowcls[a / s.nbj] * nck + s.colcls[a % s.nbj] < s.rowcls[b / s.nbj] * nck + s.colcls[b % s.nbj];
    });
    const int cs = (n + XCD_RANGES - 1) / XCD_RANGES;
    std::vector<int> order((size_t)cs * XCD_RANGES, -1);
    for (int x = 0; x < XCD_RANGES; ++x)
        for (int i = 0; i < cs && x * cs + i < n; ++i) order[(size_t)i * XCD_RANGES + x] = win[x * cs + i];
    return order;
}

// Dense C of every class of a size set (eq. (14), FP64), built on the device
// from the class tables on first use; refused with LJSDE_ENOMEM when it would
// not fit in the free device memory with 1 GiB to spare.
static int ensure_dense(Plan &p, SizeSet &s, void *stream) {
    if (s.d_dense) return LJSDE_OK;
    if (!s.d_order) {
        const std::vector<int> order = dense_order(s);
        int *d = nullptr;
        int st = dev_alloc((void **)&d, order.size() * sizeof(int));
        if (st) return st;
        const hipError_t e = hipMemcpy(d, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(LJSDE_EHIP, "dense launch order upload: %s", hipGetErrorString(e));
        }
        s.d_order = d;
        s.order_len = (int)order.size();
    }
    const size_t bytes = dense_c_bytes(p.Ws, s.n_classes());
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    if (bytes + (1ull << 30) > free_b)
        return fail(LJSDE_ENOMEM, "dense C needs %.1f GiB for %d classes, %.1f GiB free", bytes / 1073741824.0,
                    s.n_classes(), free_b / 1073741824.0);
    void *c = nullptr;
    int st = dev_alloc(&c, bytes);
    if (st) return st;
    int e = launch_dense_c_build(make_params(p), s.d_tables, s.n_classes(), p.Ws, c, stream);
    // complete before it is published: then any call, on any stream, can read it
    if (!e) e = (int)hipStreamSynchronize((hipStream_t)stream);
    if (e) {
        (void)hipFree(c);
        return fail(LJSDE_EHIP, "dense C build: %s", hipGetErrorString((hipError_t)e));
    }
    s.d_dense = c;
    return LJSDE_OK;
}

// One launch of the dense form over the windows of many images (plans of
// the dense form with equal window, block, iterations, rho, gamma, energy
// floor, pixel shape and output type). Windows are sorted by class inside
// each image, the images' lists concatenated and cut into XCD_RANGES chunks
// as for one image (workgroup b runs entry b / XCD_RANGES of chunk
// b % XCD_RANGES), so an XCD works through the classes of a few images.
static int run_dense_batch(const ljsde_job *jobs, int n, void *stream) {
    Plan *p0 = nullptr;
    int st = get_plan(jobs[0].pattern_id, &p0);
    if (st) return st;
    std::ostringstream key;
    for (int i = 0; i < n; ++i) {
        Plan *p = nullptr;
        st = get_plan(jobs[i].pattern_id, &p);
        if (st) return st;
        if (!(p->flags & LJSDE_DENSE_C))
            return fail(LJSDE_EINVAL, "job %d: a batch of the dense form needs dense-form plans only", i);
        if (p->W != p0->W || p->B != p0->B || p->iters != p0->iters || p->gamma != p0->gamma ||
            p->rho != p0->rho || p->tau != p0->tau || p->shape != p0->shape || p->fp64() != p0->fp64())
            return fail(LJSDE_EINVAL, "job %d: all plans of a dense batch need equal window, block, iters, rho, "
                                      "gamma, energy floor, pixel shape and precision", i);
        if (!jobs[i].measurements || !jobs[i].out) return fail(LJSDE_EINVAL, "job %d: null device pointer", i);
        st = check_size(*p, jobs[i].sensor_rows, jobs[i].sensor_cols);
        if (st) return st;
        key << jobs[i].pattern_id << ':' << jobs[i].sensor_rows << 'x' << jobs[i].sensor_cols << ';';
    }
    int dev = 0;
    st = current_device(&dev);
    if (st) return st;
    key << "@" << dev << "/s" << (uintptr_t)stream;
    auto &slot = g_dense_batches[key.str()];
    if (!slot) {
        auto b = std::make_unique<DenseBatch>();
        std::vector<int> list;  // (job, window) pairs
        for (int i = 0; i < n; ++i) {
            Plan *p = nullptr;
            get_plan(jobs[i].pattern_id, &p);
            SizeSet *sz = nullptr;
            if ((st = get_size(*p, jobs[i].sensor_rows, jobs[i].sensor_cols, &sz)) || (st = ensure_device(*p, *sz)) ||
                (st = ensure_dense(*p, *sz, stream))) {
                g_dense_batches.erase(key.str());
                return st;
            }
            KJob j = make_job(*p, *sz, nullptr, nullptr, nullptr, 0);
            j.dense = sz->d_dense;
            b->host_jobs.push_back(j);
            const int nw = sz->nbi * sz->nbj, nck = (int)sz->colkeys.size();
            std::vector<int> win(nw);
            for (int w = 0; w < nw; ++w) win[w] = w;
            std::stable_sort(win.begin(), win.end(), [&](int a, int c) {
                return sz->rowcls[a / sz->nbj] * nck + sz->colcls[a % sz->nbj] <
                       sz->rowcls[c / sz->nbj] * nck + sz->colcls[c % sz->nbj];
            });
            for (int w : win) {
                list.push_back(i);
                list.push_back(w);
            }
        }
        const int total = (int)(list.size() / 2);
        const int cs = (total + XCD_RANGES - 1) / XCD_RANGES;
        std::vector<int> order((size_t)cs * XCD_RANGES * 2, -1);
        for (int x = 0; x < XCD_RANGES; ++x)
            for (int i = 0; i < cs && x * cs + i < total; ++i) {
                order[((size_t)i * XCD_RANGES + x) * 2] = list[(size_t)(x * cs + i) * 2];
                order[((size_t)i * XCD_RANGES + x) * 2 + 1] = list[(size_t)(x * cs + i) * 2 + 1];
            }
        b->n_order = cs * XCD_RANGES;
        b->params = make_params(*p0);
        b->ws = p0->Ws;
        b->f32io = !p0->fp64();
        if ((st = dev_alloc((void **)&b->d_jobs, sizeof(KJob) * n)) ||
            (st = dev_alloc((void **)&b->d_order, sizeof(int) * std::max<size_t>(order.size(), 2)))) {
            g_dense_batches.erase(key.str());
            return st;
        }
        const hipError_t e = hipMemcpy(b->d_order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            g_dense_batches.erase(key.str());
            return fail(LJSDE_EHIP, "dense batch order upload: %s", hipGetErrorString(e));
        }
        slot = std::move(b);
    }
    DenseBatch *b = slot.get();
    bool changed = false;
    for (int i = 0; i < n; ++i) {
        KJob &j = b->host_jobs[i];
        if (j.y != jobs[i].measurements || j.out != jobs[i].out) {
            j.y = jobs[i].measurements;
            j.out = jobs[i].out;
            changed = true;
        }
    }
    if (changed) {
        for (int i = 0; i < n; ++i) {
            if ((st = check_device_buffer(jobs[i].measurements, "measurements", i)) ||
                (st = check_device_buffer(jobs[i].out, "out", i))) {
                for (int k = 0; k < n; ++k) b->host_jobs[k].y = b->host_jobs[k].out = nullptr;  // re-check next call
                return st;
            }
        }
        if (stream) HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        HIP_TRY(hipMemcpy(b->d_jobs, b->host_jobs.data(), sizeof(KJob) * n, hipMemcpyHostToDevice));
    }
    const int e = launch_dense_batch(b->params, b->d_jobs, b->d_order, b->n_order, b->ws, b->f32io, stream);
    if (e) return fail(LJSDE_EHIP, "dense batch launch: %s", hipGetErrorString((hipError_t)e));
    return ok();
}

// Window groups of plain L-JSDE: windows sorted by class (row-major inside
// a class), cut into groups of up to LGROUP windows of one class, and dealt so
// that workgroup b runs group b / XCD_RANGES of chunk b % XCD_RANGES of that
// list (workgroups go to the XCDs round-robin): each XCD works through a few
// classes at a time and their basis responses stay in its L2.
static std::vector<LGroup> lplain_groups(const SizeSet &s) {
    const int n = s.nbi * s.nbj, nck = (int)s.colkeys.size();
    auto cls_of = [&](int w) { return s.rowcls[w / s.nbj] * nck + s.colcls[w % s.nbj]; };
    std::vector<int> win(n);
    for (int i = 0; i < n; ++i) win[i] = i;
    std::stable_sort(win.begin(), win.end(), [&](int a, int b) { return cls_of(a) < cls_of(b); });
    std::vector<LGroup> list;
    for (int i = 0; i < n;) {
        LGroup g{};
        g.cls = cls_of(win[i]);
        while (i < n && g.count < LGROUP && cls_of(win[i]) == g.cls) g.win[g.count++] = win[i++];
        for (int k = g.count; k < LGROUP; ++k) g.win[k] = g.win[0];
        list.push_back(g);
    }
    const int ng = (int)list.size();
    const int cs = (ng + XCD_RANGES - 1) / XCD_RANGES;
    std::vector<LGroup> order((size_t)cs * XCD_RANGES);  // count 0: idle
    for (int x = 0; x < XCD_RANGES; ++x)
        for (int i = 0; i < cs && x * cs + i < ng; ++i) order[(size_t)i * XCD_RANGES + x] = list[x * cs + i];
    return order;
}

// Basis responses and normalisers of plain L-JSDE for every class of a size
// set, built on the device on first use; LJSDE_ENOMEM when they would not fit
// in the free device memory with 1 GiB to spare.
static int ensure_lplain(Plan &p, SizeSet &s, void *stream) {
    if (s.d_la) return LJSDE_OK;
    if (!s.d_lgroups) {
        const std::vector<LGroup> order = lplain_groups(s);
        LGroup *d = nullptr;
        int st = dev_alloc((void **)&d, order.size() * sizeof(LGroup));
        if (st) return st;
        const hipError_t e = hipMemcpy(d, order.data(), order.size() * sizeof(LGroup), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(LJSDE_EHIP, "L-JSDE group upload: %s", hipGetErrorString(e));
        }
        s.d_lgroups = d;
        s.n_lgroups = (int)order.size();
    }
    const size_t abytes = lplain_a_bytes(p.Ws, s.n_classes()), xbytes = lplain_aux_bytes(p.Ws, s.n_classes());
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    if (abytes + xbytes + (1ull << 30) > free_b)
        return fail(LJSDE_ENOMEM, "plain L-JSDE needs %.1f GiB of basis responses for %d classes, %.1f GiB free",
                    (abytes + xbytes) / 1073741824.0, s.n_classes(), free_b / 1073741824.0);
    void *a = nullptr, *x = nullptr;
    int st = dev_alloc(&a, abytes);
    if (st) return st;
    st = dev_alloc(&x, xbytes);
    if (st) {
        (void)hipFree(a);
        return st;
    }
    const int e = launch_lplain_build(make_params(p), s.d_tables, s.n_classes(), p.Ws, a, x, stream);
    if (e) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipFree(a);
        (void)hipFree(x);
        return fail(LJSDE_EHIP, "L-JSDE basis build: %s", hipGetErrorString((hipError_t)e));
    }
    s.d_la = a;
    s.d_laux = x;
    return LJSDE_OK;
}

static int reconstruct_impl(const void *y, int Ms, int Ns, int id, void *out, int16_t *sel, void *stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(id, &p);
    if (st) return st;
    if (!y || !out) return fail(LJSDE_EINVAL, "null device pointer");
    SizeSet *s = nullptr;
    st = get_size(*p, Ms, Ns, &s);
    if (st) return st;
    st = ensure_device(*p, *s);
    if (st) return st;
    if ((st = check_device_buffer(y, "measurements", -1)) || (st = check_device_buffer(out, "out", -1)) ||
        (sel && (st = check_device_buffer(sel, "selections", -1))))
        return st;
    KParams k = make_params(*p);
    KJob j = make_job(*p, *s, y, out, sel, 0);
    int e = 0;
    if (p->flags & LJSDE_PLAIN_L) {
        st = ensure_lplain(*p, *s, stream);
        if (st) return st;
        e = launch_lplain(k, j, s->d_la, s->d_laux, s->d_lgroups, s->n_lgroups, p->Ws, !p->fp64(), stream);
    } else if (p->flags & LJSDE_DENSE_C) {
        st = ensure_dense(*p, *s, stream);
        if (st) return st;
        e = launch_dense(k, j, s->d_dense, s->d_order, s->order_len, p->Ws, !p->fp64(), stream);
    } else if (p->fp64()) {
        e = launch_plain_f64(k, j, p->Ws, stream);
    } else if (sel) {
        e = (p->flags & LJSDE_STATE_FP32) ? launch_plain_f32(k, j, p->Ws, stream)
                                          : launch_mixed_window(k, j, p->Ws, stream);
    } else {
        ljsde_job job{y, Ms, Ns, id, out};
        return run_batch(&job, 1, stream);
    }
    if (e) return fail(LJSDE_EHIP, "kernel launch: %s", hipGetErrorString((hipError_t)e));
    return ok();
}

int ljsde_reconstruct(const void *measurements, int sensor_rows, int sensor_cols, int pattern_id, void *out,
                      void *stream) {
    return reconstruct_impl(measurements, sensor_rows, sensor_cols, pattern_id, out, nullptr, stream);
}

int ljsde_reconstruct_diag(const void *measurements, int sensor_rows, int sensor_cols, int pattern_id,
                           void *out, int16_t *selections, void *stream) {
    if (!selections) return fail(LJSDE_EINVAL, "selections is null");
    return reconstruct_impl(measurements, sensor_rows, sensor_cols, pattern_id, out, selections, stream);
}

int ljsde_reconstruct_batch(const ljsde_job *jobs, int n_jobs, void *stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (jobs && n_jobs > 0) {
        Plan *p0 = nullptr;
        const int st = get_plan(jobs[0].pattern_id, &p0);
        if (st) return st;
        if (p0->flags & LJSDE_DENSE_C) return run_dense_batch(jobs, n_jobs, stream);
    }
    return run_batch(jobs, n_jobs, stream);
}

// The work memory of this call is the per-GPU device array of
// ljsde_mixed.hip, which keeps the work list of its last call: the list is
// uploaded again only when the plan, the image size or the group width
// changes. The host copy of a list stays with the plan's size set.
int ljsde_reconstruct_noalloc(const void *measurements, int sensor_rows, int sensor_cols, int pattern_id,
                              void *out, void *stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    if (p->fp64() || (p->flags & (LJSDE_DENSE_C | LJSDE_STATE_FP32 | LJSDE_PLAIN_L)))
        return fail(LJSDE_EUNSUPPORTED, "ljsde_reconstruct_noalloc needs an FP32 plan of the factorised form "
                                        "(not LJSDE_FP64, LJSDE_DENSE_C, LJSDE_STATE_FP32 or LJSDE_PLAIN_L)");
    if (!measurements || !out) return fail(LJSDE_EINVAL, "null device pointer");
    st = check_size(*p, sensor_rows, sensor_cols);
    if (st) return st;
    const long long nwin = (long long)(2 * sensor_rows / p->B) * (2 * sensor_cols / p->B);
    if (nwin > 4LL * NOALLOC_MAX_GROUPS)
        return fail(LJSDE_EINVAL, "%dx%d sensor: %lld windows exceed the work memory of ljsde_reconstruct_noalloc "
                                  "(%d groups of at most 4 windows)", sensor_rows, sensor_cols, nwin,
                    NOALLOC_MAX_GROUPS);
    auto it = p->sizes.find(std::make_pair(sensor_rows, sensor_cols));
    if (it == p->sizes.end() || !it->second->d_tables)
        return fail(LJSDE_EINVAL, "plan %d has no device tables for a %dx%d sensor: reconstruct one image of "
                                  "that size with the plan first (ljsde_reconstruct or a batch builds them)",
                    pattern_id, sensor_rows, sensor_cols);
    SizeSet &s = *it->second;
    int dev = 0;
    st = current_device(&dev);
    if (st) return st;
    if (s.device != dev)
        return fail(LJSDE_EUNSUPPORTED, "plan tables live on device %d, current device is %d", s.device, dev);
    if ((st = check_device_buffer(measurements, "measurements", -1)) || (st = check_device_buffer(out, "out", -1)))
        return st;
    // the launch variant the autotuner chose for this shape, else the default
    TuneChoice c = default_choice(false);
    load_tune_cache();
    auto t = g_tuned.find(tune_key(*p, false, nwin, s.n_classes()));
    if (t != g_tuned.end()) c = t->second;
    forced_variant(&c);
    const int nw = c.waves_per_block;
    SizeSet::GroupList &gl = s.noalloc_lists[nw];
    if (gl.groups.empty()) make_group_list({&s}, nw, gl.groups, gl.ranges);
    if (gl.groups.size() > (size_t)NOALLOC_MAX_GROUPS)
        return fail(LJSDE_EINVAL, "%dx%d sensor: %zu window groups exceed the work memory of "
                                  "ljsde_reconstruct_noalloc (%d groups)", sensor_rows, sensor_cols,
                    gl.groups.size(), NOALLOC_MAX_GROUPS);
    int grid = 0;
    st = grid_for_shape(p->Ws, false, c, &grid);
    if (st) return st;
    unsigned char *scr = nullptr;
    int e = noalloc_scratch(dev, &scr);
    if (e) return fail(LJSDE_EHIP, "work memory address: %s", hipGetErrorString((hipError_t)e));
    // what the device array holds: (plan, sensor rows, sensor cols, group width) per device
    static int loaded[64][4];
    static bool valid[64];
    const int key[4] = {pattern_id, sensor_rows, sensor_cols, nw};
    const bool upload = !(dev < 64 && valid[dev] && std::equal(key, key + 4, loaded[dev]));
    const KParams k = make_params(*p);
    const KJob j = make_job(*p, s, measurements, out, nullptr, 0);
    if (dev < 64) valid[dev] = false;
    e = launch_mixed_noalloc(k, j, gl.groups.data(), (int)gl.groups.size(), gl.ranges, upload, p->Ws,
                             mixed_variant(c), grid, scr, stream);
    if (e) return fail(LJSDE_EHIP, "allocation-free launch: %s", hipGetErrorString((hipError_t)e));
    if (dev < 64) {
        std::copy(key, key + 4, loaded[dev]);
        valid[dev] = true;
    }
    return ok();
}

int ljsde_autotune(const ljsde_job *jobs, int n_jobs, void *stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    BatchState *b = nullptr;
    int st = prepare_batch(jobs, n_jobs, stream, &b);
    if (st) return st;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    TuneChoice best = b->choice;
    // the candidates rebuild the work list, which the captured graph refers
    // to: drop the graph now (the next batched call re-captures it for the
    // batch's choice, also when the tuning fails part-way)
    (void)hipStreamSynchronize((hipStream_t)stream);
    drop_graph(*b);
    auto time_one = [&](const TuneChoice &c) -> int {
        int grid = 0;
        int st2 = grid_for(*b, c, &grid);
        if (st2) return st2;
        if (!b->state_fp32) {
            st2 = build_groups(*b, c.waves_per_block);
            if (st2) return st2;
        }
        // warm-up, also timed: short launches are repeated until a candidate
        // has run for about 30 ms, so that launch jitter does not pick it
        (void)hipEventRecord(e0, (hipStream_t)stream);
        st2 = launch_batch_eager(*b, c, grid, stream);
        if (st2) return st2;
        (void)hipEventRecord(e1, (hipStream_t)stream);
        hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) return fail(LJSDE_EHIP, "autotune: %s", hipGetErrorString(e));
        float total = 0;
        (void)hipEventElapsedTime(&total, e0, e1);
        const int reps = std::max(3, std::min(50, (int)(30.0f / std::max(total, 1e-3f))));
        (void)hipEventRecord(e0, (hipStream_t)stream);
        for (int r = 0; r < reps && !st2; ++r) st2 = launch_batch_eager(*b, c, grid, stream);
        (void)hipEventRecord(e1, (hipStream_t)stream);
        if (st2) return st2;
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) return fail(LJSDE_EHIP, "autotune: %s", hipGetErrorString(e));
        (void)hipEventElapsedTime(&total, e0, e1);
        if (total / reps < best_ms) {
            best_ms = total / reps;
            best = c;
        }
        return LJSDE_OK;
    };
    if (b->state_fp32) {
        for (const TuneChoice &c : std::vector<TuneChoice>{
                 {1, 1}, {1, 2}, {1, 4}, {1, 8}, {2, 2}, {2, 4}, {4, 2}, {4, 4}})
            if ((st = time_one(c))) break;
    } else {
        // stage 1: windows per workgroup and resident workgroups per CU;
        // stage 2: groups per claim; stage 3: the LDS layout of the per-lane
        // tables and the DFT tile shape (W = 32 without split-BF16 only)
        for (const TuneChoice &c : std::vector<TuneChoice>{{1, 1, 0}, {2, 1, 0}, {4, 1, 0}, {2, 1, 1}, {4, 1, 1}})
            if ((st = time_one(c))) break;
        if (!st) {
            const TuneChoice base = best;
            for (int chunk : {2, 4}) {
                TuneChoice c = base;
                c.chunk = chunk;
                if ((st = time_one(c))) break;
            }
        }
        if (!st && b->ws == 16 && !b->params.dft_bf16) {
            const TuneChoice base = best;
            TuneChoice c = base;
            c.qreg = 1;
            st = time_one(c);
            if (!st) {
                c = base;
                c.vdft = 1;
                st = time_one(c);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    b->choice = best;
    g_tuned[b->tune_key] = best;
    save_tune_cache();
    st = capture_graph(*b);
    if (st) return st;
    return ok();
}

int ljsde_synchronize(void *stream) {
    int dev = 0;
    int st = current_device(&dev);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipGetLastError());
    return ok();
}

int ljsde_release(int pattern_id) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    // work in flight may still read the plan's tables
    if (p->d_consts) (void)hipDeviceSynchronize();
    // batches that reference this plan hold device pointers into its tables
    drop_batches_of(pattern_id);
    for (auto &kv : p->sizes) {
        SizeSet &s = *kv.second;
        if (s.d_tables) (void)hipFree(s.d_tables);
        if (s.d_rowcls) (void)hipFree(s.d_rowcls);
        if (s.d_colcls) (void)hipFree(s.d_colcls);
        if (s.d_dense) (void)hipFree(s.d_dense);
        if (s.d_order) (void)hipFree(s.d_order);
        if (s.d_la) (void)hipFree(s.d_la);
        if (s.d_laux) (void)hipFree(s.d_laux);
        if (s.d_lgroups) (void)hipFree(s.d_lgroups);
    }
    if (p->d_consts) (void)hipFree(p->d_consts);
    g_plans[pattern_id].reset();
    return ok();
}

int ljsde_class_count(int pattern_id, int sensor_rows, int sensor_cols, int32_t *class_of_window) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    SizeSet *s = nullptr;
    st = get_size(*p, sensor_rows, sensor_cols, &s);
    if (st) return st;
    if (class_of_window) {
        const int nck = (int)s->colkeys.size();
        for (int bi = 0; bi < s->nbi; ++bi)
            for (int bj = 0; bj < s->nbj; ++bj)
                class_of_window[(size_t)bi * s->nbj + bj] = s->rowcls[bi] * nck + s->colcls[bj];
    }
    ok();
    return s->n_classes();
}

int ljsde_class_tables(int pattern_id, int sensor_rows, int sensor_cols, int class_index, double *S, double *D,
                       int8_t *codes) {
    std::lock_guard<std::mutex> lk(g_mu);
    Plan *p = nullptr;
    int st = get_plan(pattern_id, &p);
    if (st) return st;
    SizeSet *s = nullptr;
    st = get_size(*p, sensor_rows, sensor_cols, &s);
    if (st) return st;
    if (class_index < 0 || class_index >= s->n_classes())
        return fail(LJSDE_EINVAL, "class %d out of range [0, %d)", class_index, s->n_classes());
    build_host_tables(*p, *s);
    const unsigned char *blk = s->blob.data() + (size_t)class_index * p->lay.stride;
    if (S) memcpy(S, blk + p->lay.offS, sizeof(double) * p->Ws * p->Ws * 2 * p->n_spectra());
    if (D) memcpy(D, s->D.data() + (size_t)class_index * p->W * p->W, sizeof(double) * p->W * p->W);
    if (codes) memcpy(codes, blk + p->lay.offCodes, p->Ws * p->Ws);
    return ok();
}

}  // extern "C"
