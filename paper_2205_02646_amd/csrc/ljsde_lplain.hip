// Plain L-JSDE (Sec. III; Sec. IV eqs. (4)-(10), (15), (16); eq. (18)) on gfx950.
//
// This is the method before its recurrence is exploited. Each window keeps
// its weighted residual x_m = w_m r_m in the measurement domain (eq. (7)) and
// re-evaluates the numerator of eq. (10) for every basis function in every
// iteration,
//     R(f) = sum_m w_m r_m conj(a_m(f)),  a_m(f) = sum_{eta, gamma} A_m(eta, gamma) Phi(eta, gamma, f),
// a dense product of the W^2 x (W/2)^2 matrix conj(a)^T with the residual:
// O(W^4) work per iteration, against O(W^2) for RL-JSDE. The step and the
// residual update follow eqs. (15), (16) and (7): r -= gamma delta a(:, k).
//
// Windows whose local measurement matrices are equal have equal a, so one
// workgroup runs up to LGROUP = 16 such windows in lockstep and the product
// becomes a complex GEMM [W^2 x (W/2)^2] x [(W/2)^2 x 16] on FP64 MFMA
// (v_mfma_f64_16x16x4f64): frequencies on the rows, windows on the columns,
// the local sensor pixels m as the contraction. The four wavefronts split the
// frequencies; the residuals of the 16 windows sit in LDS (64 KiB at W = 32),
// and a streams from L2 in the layout the MFMA's A operand reads
// ([tile of 16 frequencies][m][16 frequencies], 1 KiB per wavefront load).
//
// a is built on the device from A and Phi as the definition writes it (a sum
// over the quadrants each sensor pixel integrates, or weighs for general
// layouts), and D of eq. (10) from a. A window that has no other window of
// its class (a non-recurrent pattern) runs alone in its workgroup: the same
// product with 15 empty columns.
#include <hip/hip_runtime.h>

#include "ljsde_device.h"
#include "ljsde_internal.h"

namespace ljsde {

// A frequency whose D of eq. (10) is at most L_D_REL of the class's largest
// D has no response in the window (its D is 0 in exact arithmetic): metric 0,
// never selected, and no step (the same threshold as the class tables).
constexpr double L_D_REL = 1e-13;

size_t lplain_a_bytes(int ws, int n_classes) {
    const size_t W = 2 * (size_t)ws;
    return (size_t)n_classes * W * W * (size_t)ws * ws * 16;
}

size_t lplain_aux_bytes(int ws, int n_classes) {
    const size_t W = 2 * (size_t)ws;
    return (size_t)n_classes * 2 * W * W * sizeof(double);
}

// Basis responses of every class: a[((cls * NT + t) * NPOS + m) * 16 + fl] =
// a_m(16 t + fl). Grid (NT = W^2 / 16 tiles, classes); one thread per local
// sensor pixel m = (W/2) i' + j', whose footprint is rows 2i', 2i' + 1 and
// columns 2j', 2j' + 1 of the window.
template <int WS>
__global__ __launch_bounds__(WS *WS) void lplain_a_kernel(KParams p, const unsigned char *tables, double2 *a) {
    constexpr int W = 2 * WS, NPOS = WS * WS, NT = W * W / 16;
    const int t = blockIdx.x, cls = blockIdx.y, m = threadIdx.x;
    const unsigned char *tb = tables + (size_t)cls * p.lay.stride;
    const int code = ((const signed char *)(tb + p.lay.offCodes))[m];
    const int ip = m / WS, jp = m % WS;
    // row m of A: the weight of quadrant q = 2 qa + qb of the pixel's footprint
    double wq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (code < 0) wq[q] = 0.0;  // absent pixel: zero row
        else if (p.shape == SHAPE_GENERAL) wq[q] = ((const double *)(tb + p.lay.offA))[m * 4 + q];
        else wq[q] = ((p.shape >> (q ^ code)) & 1) ? 1.0 : 0.0;
    }
    double2 *dst = a + (((size_t)cls * NT + t) * NPOS + m) * 16;
    for (int fl = 0; fl < 16; ++fl) {
        const int f = 16 * t + fl, s = f / W, r = f % W;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // Phi(2i' + qa, 2j' + qb, s, r) = exp(i 2 pi ((2i' + qa) s + (2j' + qb) r) / W)
            const int ph = ((2 * ip + (q >> 1)) * s + (2 * jp + (q & 1)) * r) & (W - 1);
            re += wq[q] * p.c.ew[2 * ph];
            im += wq[q] * p.c.ew[2 * ph + 1];
        }
        dst[fl] = make_double2(re, im);
    }
}

// D(f) = sum_m w_m |a_m(f)|^2 (eq. (10), w_m = 0 for absent pixels), then
// q / D and 1 / D (0 where unobserved): aux[cls][0][f], aux[cls][1][f].
// One workgroup of 256 threads per class.
template <int WS>
__global__ __launch_bounds__(256) void lplain_aux_kernel(KParams p, const unsigned char *tables, const double2 *a,
                                                         double *aux) {
    constexpr int W = 2 * WS, NPOS = WS * WS, NF = W * W, NT = NF / 16, FPT = NF / 256;
    __shared__ double red[256];
    const int cls = blockIdx.x, tid = threadIdx.x;
    const signed char *codes = (const signed char *)(tables + (size_t)cls * p.lay.stride + p.lay.offCodes);
    const double2 *A = a + (size_t)cls * NT * NPOS * 16;
    double D[FPT];
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
        const int f = tid + 256 * i;
        const double2 *col = A + (size_t)(f / 16) * NPOS * 16 + (f % 16);
        double d = 0.0;
        for (int m = 0; m < NPOS; ++m) {
            const double wm = codes[m] >= 0 ? p.c.w[m] : 0.0;
            const double2 v = col[(size_t)m * 16];
            d += wm * (v.x * v.x + v.y * v.y);
        }
        D[i] = d;
        dmax = fmax(dmax, d);
    }
    red[tid] = dmax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double thr = L_D_REL * red[0];
    double *qd = aux + (size_t)cls * 2 * NF;
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
        const int f = tid + 256 * i;
        const bool obs = D[i] > 0.0 && D[i] > thr;
        qd[f] = obs ? p.c.q[f] / D[i] : 0.0;
        qd[NF + f] = obs ? 1.0 / D[i] : 0.0;
    }
}

// Running selection of eq. (10) with the tie rule of the other kernels
// (metrics within a relative TIE_REL of the maximum count as maximal, the
// lowest frequency index wins), carrying R of the kept frequency.
struct LSel {
    double best, re, im;
    int idx;
};

__device__ __forceinline__ void lsel_keep(LSel &s, double m, int f, double re, double im) {
    // frequencies arrive in increasing order
    if (m > s.best * (1.0 + TIE_REL)) {
        s.best = m;
        s.idx = f;
        s.re = re;
        s.im = im;
    } else if (m > s.best) {
        s.best = m;  // inside the tie band: the lower index stays
    }
}

__device__ __forceinline__ void lsel_merge(LSel &s, const LSel &o) {
    if (o.best > s.best * (1.0 + TIE_REL)) {
        s = o;
    } else if (!(s.best > o.best * (1.0 + TIE_REL))) {
        s.best = fmax(s.best, o.best);
        if (o.idx < s.idx) {
            s.idx = o.idx;
            s.re = o.re;
            s.im = o.im;
        }
    }
}

__device__ __forceinline__ LSel lsel_shfl_xor(const LSel &s, int o) {
    LSel r;
    r.best = __shfl_xor(s.best, o);
    r.re = __shfl_xor(s.re, o);
    r.im = __shfl_xor(s.im, o);
    r.idx = __shfl_xor(s.idx, o);
    return r;
}

struct LStep {
    double gr, gi;  // gamma * delta of eqs. (15)-(16)
    int k;          // selected frequency
    int live;       // the window still iterates
};

// One workgroup (4 wavefronts) per group of up to LGROUP windows of one class.
// IO is the element type of the output (FP32 plans: float; the arithmetic is
// FP64 either way); the measurements are double or float by the job's flag.
template <int WS, typename IO>
__global__ __launch_bounds__(256) void lplain_kernel(KParams p, KJob j, const double2 *__restrict__ amat,
                                                     const double *__restrict__ aux,
                                                     const LGroup *__restrict__ groups) {
    constexpr int W = 2 * WS, NPOS = WS * WS, NF = W * W, NT = NF / 16, TPW = NT / 4, KS = NPOS / 4;
    static_assert(TPW % 4 == 0, "tiles per wavefront: whole passes of four");
    __shared__ double2 X[NPOS * LGROUP];  // x[m][window] = w_m r_m
    __shared__ LSel red[4 * LGROUP];
    __shared__ LStep step[LGROUP];

    const int cls = groups[blockIdx.x].cls, cnt = groups[blockIdx.x].count;
    if (cnt == 0) return;  // idle workgroup (uniform)
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned char *tb = j.tables + (size_t)cls * p.lay.stride;
    const signed char *codes = (const signed char *)(tb + p.lay.offCodes);
    const double2 *A = amat + (size_t)cls * NT * NPOS * 16;
    const double *qD = aux + (size_t)cls * 2 * NF;
    const double *invD = qD + NF;

    // ---- local measurements of the windows, weighted (absent pixels -> 0) ----
    // thread tid always handles window tid % LGROUP
    const int mywin = tid % LGROUP;
    double e0 = 0.0;
    {
        int bi = 0, bj = 0;
        if (mywin < cnt) {
            const int w = groups[blockIdx.x].win[mywin];
            bi = w / j.nbj;
            bj = w % j.nbj;
        }
        const int rs = (p.B * bi - p.off) / 2, cs = (p.B * bj - p.off) / 2;
        for (int e = tid; e < NPOS * LGROUP; e += 256) {
            const int m = e / LGROUP;
            const int gi = rs + m / WS, gj = cs + m % WS;
            double x = 0.0;
            if (mywin < cnt && codes[m] >= 0 && gi >= 0 && gi < j.Ms && gj >= 0 && gj < j.Ns) {
                const double yv = load_measurement(j, (size_t)gi * j.Ns + gj);
                x = p.c.w[m] * yv;
                e0 += x * yv;
            }
            X[e] = make_double2(x, 0.0);
        }
    }
    // E(0) of eq. (8) per window: lanes of equal lane % 16, then the wavefronts
    e0 += __shfl_xor(e0, 16);
    e0 += __shfl_xor(e0, 32);
    if (lane < LGROUP) red[wave * LGROUP + lane].best = e0;
    __syncthreads();
    double E = 0.0, E0 = 0.0;
    if (tid < LGROUP) {
        E0 = red[tid].best + red[LGROUP + tid].best + red[2 * LGROUP + tid].best + red[3 * LGROUP + tid].best;
        E = E0;
        step[tid].live = tid < cnt ? 1 : 0;
    }
    __syncthreads();

    const int BB = p.B * p.B;
    double outacc[4] = {0.0, 0.0, 0.0, 0.0};  // eq. (18): (window, pixel) pairs tid + 256 q
    int nu_done = 0;

#pragma unroll 1
    for (int nu = 0; nu < p.iters; ++nu) {
        // ---- eq. (10): R = conj(a)^T x for this wavefront's TPW frequency tiles ----
        LSel s = {-1.0, 0.0, 0.0, 0};
#pragma unroll 1
        for (int pass = 0; pass < TPW / 4; ++pass) {
            const int t0 = wave * TPW + pass * 4;
            v4f64 cr[4], ci[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cr[i] = v4f64{0.0, 0.0, 0.0, 0.0};
                ci[i] = v4f64{0.0, 0.0, 0.0, 0.0};
            }
            // lane L loads a_m(f) for m = 4 ks + L / 16, f = 16 t + L % 16 (the A
            // operand) and x[m][L % 16] (the B operand)
            const double2 *ap = A + (size_t)t0 * NPOS * 16 + lane;
#pragma unroll 2
            for (int ks = 0; ks < KS; ++ks) {
                const double2 xv = X[ks * 64 + lane];
                double2 av[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = ap[((size_t)i * NPOS + 4 * ks) * 16];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // conj(a) x = (a.re x.re + a.im x.im) + i (a.re x.im - a.im x.re)
                    cr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, xv.x, cr[i], 0, 0, 0);
                    cr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, xv.y, cr[i], 0, 0, 0);
                    ci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, xv.y, ci[i], 0, 0, 0);
                    ci[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[i].y, xv.x, ci[i], 0, 0, 0);
                }
            }
            // result: lane L, register r holds frequency 16 t + L / 16 + 4 r of
            // window L % 16 (increasing in r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = (t0 + i) * 16 + lane / 16 + 4 * r;
                    const double re = cr[i][r], im = ci[i][r];
                    lsel_keep(s, (re * re + im * im) * qD[f], f, re, im);
                }
        }
        // ---- selection per window: lanes of equal lane % 16, then the wavefronts ----
        lsel_merge(s, lsel_shfl_xor(s, 16));
        lsel_merge(s, lsel_shfl_xor(s, 32));
        if (lane < LGROUP) red[wave * LGROUP + lane] = s;
        __syncthreads();
        if (tid < LGROUP) {
            LSel b = red[tid];
#pragma unroll
            for (int w = 1; w < 4; ++w) lsel_merge(b, red[w * LGROUP + tid]);
            LStep st = step[tid];
            st.k = b.idx;
            st.gr = 0.0;
            st.gi = 0.0;
            if (st.live) {
                // eqs. (15)-(16): delta = R_k / D_k (0 at an unobserved frequency)
                const double id = invD[b.idx];
                st.gr = p.gamma * id * b.re;
                st.gi = p.gamma * id * b.im;
                E -= p.ecoef * (b.re * b.re + b.im * b.im) * id;
                if (p.tau > 0.0 && E <= p.tau * E0) st.live = 0;  // this pick still counts
            }
            if (j.sel != nullptr && tid < cnt) {
                // the pick, or -1 once the window has stopped
                const int w = groups[blockIdx.x].win[tid];
                j.sel[(size_t)w * p.iters + nu] = (int16_t)(step[tid].live ? b.idx : -1);
            }
            step[tid] = st;
        }
        __syncthreads();
        // ---- eq. (7): x -= gamma delta w a(:, k); eq. (18) pick by pick ----
        {
            const LStep st = step[mywin];
            const double2 *col = A + (size_t)(st.k / 16) * NPOS * 16 + (st.k % 16);
#pragma unroll 4
            for (int mm = 0; mm < NPOS / 16; ++mm) {
                const int m = tid / LGROUP + 16 * mm;
                const double wm = codes[m] >= 0 ? p.c.w[m] : 0.0;
                const double2 av = col[(size_t)m * 16];
                const double ar = wm * av.x, ai = wm * av.y;
                double2 xv = X[tid + 256 * mm];
                xv.x -= st.gr * ar - st.gi * ai;
                xv.y -= st.gr * ai + st.gi * ar;
                X[tid + 256 * mm] = xv;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            if (e < LGROUP * BB) {
                const LStep st = step[e / BB];
                const int px = e % BB, oi = px / p.B, oj = px % p.B;
                const int u = st.k / W, v = st.k % W;
                const int ph = ((p.off + oi) * u + (p.off + oj) * v) & (W - 1);
                outacc[q] += st.gr * p.c.ew[2 * ph] - st.gi * p.c.ew[2 * ph + 1];
            }
        }
        nu_done = nu + 1;
        __syncthreads();
        if (p.tau > 0.0) {
            int any = 0;
#pragma unroll
            for (int w = 0; w < LGROUP; ++w) any |= step[w].live;
            if (!any) break;  // every window stopped (uniform: read after the barrier)
        }
    }
    // selections after the last iteration run (every window had stopped)
    if (j.sel != nullptr)
        for (int e = tid; e < cnt * p.iters; e += 256) {
            const int w = e / p.iters, nu = e % p.iters;
            if (nu >= nu_done) j.sel[(size_t)groups[blockIdx.x].win[w] * p.iters + nu] = -1;
        }
    IO *O = (IO *)j.out;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        if (e < LGROUP * BB && e / BB < cnt) {
            const int w = groups[blockIdx.x].win[e / BB];
            const int bi = w / j.nbj, bj = w % j.nbj;
            const int px = e % BB, oi = px / p.B, oj = px % p.B;
            O[(size_t)(p.B * bi + oi) * (size_t)(2 * j.Ns) + (size_t)(p.B * bj + oj)] = (IO)outacc[q];
        }
    }
}

template <int WS>
static int launch_build(const KParams &p, const unsigned char *tables, int n_classes, void *a, void *aux,
                        void *stream) {
    constexpr int W = 2 * WS, NT = W * W / 16;
    lplain_a_kernel<WS><<<dim3(NT, n_classes), dim3(WS * WS), 0, (hipStream_t)stream>>>(p, tables, (double2 *)a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    lplain_aux_kernel<WS><<<dim3(n_classes), dim3(256), 0, (hipStream_t)stream>>>(p, tables, (const double2 *)a,
                                                                                 (double *)aux);
    return (int)hipGetLastError();
}

int launch_lplain_build(const KParams &p, const unsigned char *tables, int n_classes, int ws, void *a, void *aux,
                        void *stream) {
    if (n_classes <= 0) return 0;
    return ws == 16 ? launch_build<16>(p, tables, n_classes, a, aux, stream)
                    : launch_build<8>(p, tables, n_classes, a, aux, stream);
}

template <typename IO>
static int launch_lplain_io(const KParams &p, const KJob &job, const void *a, const void *aux, const LGroup *groups,
                            int ngroups, int ws, void *stream) {
    if (ws == 16)
        lplain_kernel<16, IO><<<dim3(ngroups), dim3(256), 0, (hipStream_t)stream>>>(p, job, (const double2 *)a,
                                                                                   (const double *)aux, groups);
    else
        lplain_kernel<8, IO><<<dim3(ngroups), dim3(256), 0, (hipStream_t)stream>>>(p, job, (const double2 *)a,
                                                                                  (const double *)aux, groups);
    return (int)hipGetLastError();
}

int launch_lplain(const KParams &p, const KJob &job, const void *a, const void *aux, const LGroup *groups,
                  int ngroups, int ws, bool f32io, void *stream) {
    if (ngroups <= 0) return 0;
    return f32io ? launch_lplain_io<float>(p, job, a, aux, groups, ngroups, ws, stream)
                 : launch_lplain_io<double>(p, job, a, aux, groups, ngroups, ws, stream);
}

}  // namespace ljsde
