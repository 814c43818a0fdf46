// HIP kernels of the RL-JSDE hot path for gfx950 (CDNA4, wave64).
//
// One wavefront models one window. The loop state is the factorised
// projected residual: for each opaque-quadrant orientation o the (W/2)-point
// 2-D DFT of the weighted residual restricted to the sensor pixels of that
// orientation,
//     P_o(k, l) = sum_{m: o_m = o} w_m r_m exp(-2 pi i (i' k + j' l) / Ws),
// from which the projected residual of eq. (12) follows for every frequency
// (sigma, rho) = (k + Ws a, l + Ws b) as
//     R(sigma, rho) = sum_o conj(H_o(sigma, rho)) P_o(k, l),
// with H_o the response of the pixel of code o to the basis function: for the
// L-shaped pixels of three-quarter sampling the box response of the 2x2
// footprint minus the opaque quadrant, for quarter sampling the response of
// the one transparent quadrant.
// Selecting (u, v) by eq. (11) and taking the step of eqs. (15)-(16) changes
// every P_o by the orientation's weighted-mask spectrum S_o shifted by (u, v)
// (eq. (17) in factorised form):
//     P_o(k, l) -= gamma delta H_o(u, v) S_o(k - u, l - v).
// S_o, q / D and 1 / D come from the per-class FP64 tables.
//
// Lane layout (Ws = 16): lane L owns the (k, l) positions
// k = 4 (L / 16) + t (t < 4), l = L % 16, i.e. 16 frequencies. The 4x4
// frequencies of one position are formed from its four P_o by a twiddle step
// and a 2x2 Walsh-Hadamard step. S_o lives in LDS; the state, the per-lane
// q / D and the twiddles live in VGPRs.
#include <hip/hip_runtime.h>

#include "ljsde_device.h"
#include "ljsde_internal.h"
#include "ljsde_window.h"

namespace ljsde {

template <typename T>
__device__ __forceinline__ T load_qd(const double *qd64, const float *qd32, int i);
template <>
__device__ __forceinline__ double load_qd<double>(const double *qd64, const float *, int i) {
    return qd64[i];
}
template <>
__device__ __forceinline__ float load_qd<float>(const double *, const float *qd32, int i) {
    return qd32[i];
}

template <typename T, int WS, int SHAPE>
__device__ __forceinline__ void process_window(const KParams &p, const KJob &j, int bi, int bj,
                                               long long win_local, char *lds) {
    constexpr int W = 2 * WS;
    constexpr int QPL = WS * WS / 64;
    constexpr int NPOS = WS * WS;
    const int lane = threadIdx.x & 63;
    // lane L owns the positions k = L / WS + KSTEP t (t < QPL), l = L % WS
    constexpr int KSTEP = 64 / WS;
    const int lam = lane % WS;
    const int krow = lane / WS;

    const int cls = j.rowcls[bi] * j.ncolk + j.colcls[bj];
    const unsigned char *tb = j.tables + (size_t)cls * p.lay.stride;
    const double *S64 = (const double *)(tb + p.lay.offS);
    const double *qD64 = (const double *)(tb + p.lay.offQD64);
    const double *invD = (const double *)(tb + p.lay.offInvD);
    const float *qD32 = (const float *)(tb + p.lay.offQD32);
    const signed char *codes = (const signed char *)(tb + p.lay.offCodes);

    T *ldsS = (T *)lds;                 // stage buffer, then S_o: [o][pos][re, im]
    T *ldsX = ldsS + NPOS * 8;          // weighted measurements w_m y_m
    signed char *ldsC = (signed char *)(ldsX + NPOS);
    C2<T> P[QPL][4];
    const double e0 = window_prologue<T, WS>(p, j, bi, bj, codes, ldsX, ldsC, ldsS, P);

    // ---- class spectra S_o into LDS (FP64 table -> working precision) ------
    // table order [pos][o][re, im] -> LDS order [o][pos][re, im] (bank-conflict-free reads)
    for (int e = lane; e < NPOS * 8; e += 64) ldsS[((((e >> 1) & 3) * NPOS) + (e >> 3)) * 2 + (e & 1)] = (T)S64[e];

    // ---- per-lane constants -------------------------------------------------
    T qd[QPL][4];
    C2<T> tk[QPL], tkl[QPL];
#pragma unroll
    for (int t = 0; t < QPL; ++t) {
        const int kap = krow + KSTEP * t;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                qd[t][a * 2 + b] = load_qd<T>(qD64, qD32, (kap + WS * a) * W + lam + WS * b);
        tk[t] = {(T)p.c.ew[2 * kap], (T)-p.c.ew[2 * kap + 1]};
        tkl[t] = {(T)p.c.ew[2 * (kap + lam)], (T)-p.c.ew[2 * (kap + lam) + 1]};
    }
    const C2<T> tl = {(T)p.c.ew[2 * lam], (T)-p.c.ew[2 * lam + 1]};
    wave_lds_fence();

    const int BB = p.B * p.B;
    const int oi = lane / p.B, oj = lane % p.B;
    double outacc = 0.0;
    double E = e0;
    C2<T> g4[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) g4[o] = {T(0), T(0)};
    int u = 0, v = 0;
    int nu_done = 0;
    // FP64: ties within TIE_REL go to the lowest index; the FP32 state
    // variant compares strictly (its rounding is far above TIE_REL)
    const T eps = sizeof(T) == 8 ? T(TIE_REL) : T(0);

#pragma unroll 1
    for (int nu = 0; nu < p.iters; ++nu) {
        // issue priority: the update and projection at 0, the dependent chain
        // from the selection to the step at 2, so that of the wavefronts of a
        // SIMD the one in that chain issues first
        __builtin_amdgcn_s_setprio(0);
        T m[QPL][4];
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
            const int kap = krow + KSTEP * t;
            if (nu > 0) {
                // subtract the shifted weighted-mask spectra of the last pick
                const int pos = ((kap - u) & (WS - 1)) * WS + ((lam - v) & (WS - 1));
                const T *s = ldsS + pos * 2;
#pragma unroll
                for (int o = 0; o < 4; ++o) {  // two fused multiply-adds per component
                    const T sr = s[o * NPOS * 2], si = s[o * NPOS * 2 + 1];
                    P[t][o].re = fma(-g4[o].re, sr, fma(g4[o].im, si, P[t][o].re));
                    P[t][o].im = fma(-g4[o].re, si, fma(-g4[o].im, sr, P[t][o].im));
                }
            }
            // project: R(a, b) = sum_q (-1)^(qa a + qb b) e^{-i theta (qa k + qb l)} Q_q with the
            // per-quadrant sums of the pixel shape (sum P - P_q for three-quarter sampling)
            C2<T> Q[4];
            shape_sums<SHAPE, T>(P[t], Q);
            const C2<T> q0 = Q[0], q1 = Q[1], q2 = Q[2], q3 = Q[3];
            const C2<T> u1 = {tl.re * q1.re - tl.im * q1.im, tl.re * q1.im + tl.im * q1.re};
            const C2<T> u2 = {tk[t].re * q2.re - tk[t].im * q2.im, tk[t].re * q2.im + tk[t].im * q2.re};
            const C2<T> u3 = {tkl[t].re * q3.re - tkl[t].im * q3.im,
                              tkl[t].re * q3.im + tkl[t].im * q3.re};
            const C2<T> s1 = {q0.re + u3.re, q0.im + u3.im}, d1 = {q0.re - u3.re, q0.im - u3.im};
            const C2<T> s2 = {u1.re + u2.re, u1.im + u2.im}, d2 = {u1.re - u2.re, u1.im - u2.im};
            const C2<T> r00 = {s1.re + s2.re, s1.im + s2.im};
            const C2<T> r01 = {d1.re - d2.re, d1.im - d2.im};
            const C2<T> r10 = {d1.re + d2.re, d1.im + d2.im};
            const C2<T> r11 = {s1.re - s2.re, s1.im - s2.im};
            // eq. (11) metric q |R|^2 / D
            m[t][0] = (r00.re * r00.re + r00.im * r00.im) * qd[t][0];
            m[t][1] = (r01.re * r01.re + r01.im * r01.im) * qd[t][1];
            m[t][2] = (r10.re * r10.re + r10.im * r10.im) * qd[t][2];
            m[t][3] = (r11.re * r11.re + r11.im * r11.im) * qd[t][3];
        }
        // first maximum in sigma * W + rho order (within the tie band)
        __builtin_amdgcn_s_setprio(2);
        const int idx = select_lowest_max<T, WS, QPL>(m, eps, lane);
        u = idx / W;
        v = idx % W;

        // L-pixel responses of the selected basis function (FP64 table)
        const double *Hp = p.c.H + (size_t)idx * 8;  // uniform index: scalar loads
        double Hr[4], Hi[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            Hr[o] = Hp[2 * o];
            Hi[o] = Hp[2 * o + 1];
        }

        // R_uv in FP64 from the owner lane's state
        const int ku = u & (WS - 1), lv = v & (WS - 1);
        const int tu = ku / KSTEP;
        const int owner = (ku % KSTEP) * WS + lv;
        C2<T> Pu[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) Pu[o] = P[0][o];
#pragma unroll
        for (int t = 1; t < QPL; ++t)
            if (tu == t) {
#pragma unroll
                for (int o = 0; o < 4; ++o) Pu[o] = P[t][o];
            }
        double rr = 0.0, ri = 0.0;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const double pr = (double)Pu[o].re, pi = (double)Pu[o].im;
            rr += Hr[o] * pr + Hi[o] * pi;
            ri += Hr[o] * pi - Hi[o] * pr;
        }
        rr = readlane_f64(rr, owner);
        ri = readlane_f64(ri, owner);

        // eqs. (15)-(16): delta = R_uv / D_uv, step gamma * delta; energy in FP64
        const double id = invD[idx];
        const double gr = p.gamma * rr * id, gi = p.gamma * ri * id;
        E -= p.ecoef * (rr * rr + ri * ri) * id;
#pragma unroll
        for (int o = 0; o < 4; ++o)
            g4[o] = {(T)(gr * Hr[o] - gi * Hi[o]), (T)(gr * Hi[o] + gi * Hr[o])};

        // eq. (18) restricted to the central block, accumulated pick by pick
        if (lane < BB) {
            const int ph = ((p.off + oi) * u + (p.off + oj) * v) & (W - 1);
            outacc += gr * p.c.ew[2 * ph] - gi * p.c.ew[2 * ph + 1];
        }
        if (j.sel != nullptr && lane == 0) j.sel[win_local * p.iters + nu] = (int16_t)idx;
        nu_done = nu + 1;
        if (p.tau > 0.0 && E <= p.tau * e0) break;
    }
    if (j.sel != nullptr)
        for (int nu = nu_done + lane; nu < p.iters; nu += 64) j.sel[win_local * p.iters + nu] = -1;

    if (lane < BB) {
        T *O = (T *)j.out;
        const size_t row = (size_t)(p.B * bi + oi);
        O[row * (size_t)(2 * j.Ns) + (size_t)(p.B * bj + oj)] = (T)outacc;
    }
}

// occupancy targets: 2 wavefronts per SIMD in FP64 (state 64 VGPRs alone),
// 3 with the FP32 state
template <typename T>
struct Occ {
    static constexpr int waves = sizeof(T) == 8 ? 2 : 3;
};

template <typename T, int WS, int SHAPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Occ<T>::waves))) void plain_kernel(KParams p,
                                                                                                        KJob j) {
    extern __shared__ char lds[];
    const long long w = blockIdx.x;
    const long long nwin = (long long)j.nbi * j.nbj;
    if (w >= nwin) return;
    process_window<T, WS, SHAPE>(p, j, (int)(w / j.nbj), (int)(w % j.nbj), w, lds);
}

__global__ void reset_counter_kernel(unsigned int *counters) {
    if (blockIdx.x == 0 && threadIdx.x < COUNTERS) counters[threadIdx.x] = 0u;
}

template <typename T, int WS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void persistent_kernel(KParams p, const KJob *__restrict__ jobs,
                                                         int njobs, long long total,
                                                         unsigned int *counter, int chunk) {
    extern __shared__ char lds[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    char *mylds = lds + (size_t)wave * WinLds<T, WS>::bytes;
    for (;;) {
        unsigned int start = 0;
        if (lane == 0) start = atomicAdd(counter, (unsigned int)chunk);
        start = __shfl(start, 0);
        start = __builtin_amdgcn_readfirstlane(start);
        if ((long long)start >= total) break;
        const long long end = min((long long)start + chunk, total);
        for (long long gw = start; gw < end; ++gw) {
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].win_begin <= gw) lo = mid;
                else hi = mid - 1;
            }
            const KJob j = jobs[lo];
            const long long lw = gw - j.win_begin;
            process_window<T, WS, SHAPE_THREE_QUARTER>(p, j, (int)(lw / j.nbj), (int)(lw % j.nbj), lw, mylds);
        }
    }
}

size_t lds_bytes_per_wave(int ws, bool fp64) {
    if (ws == 16) return fp64 ? WinLds<double, 16>::bytes : WinLds<float, 16>::bytes;
    return fp64 ? WinLds<double, 8>::bytes : WinLds<float, 8>::bytes;
}

template <typename T, int WS, int SHAPE>
static int launch_plain_t(const KParams &p, const KJob &job, void *stream) {
    const long long nwin = (long long)job.nbi * job.nbj;
    if (nwin <= 0) return 0;
    const size_t lds = WinLds<T, WS>::bytes;
    plain_kernel<T, WS, SHAPE><<<dim3((unsigned)nwin), dim3(64), lds, (hipStream_t)stream>>>(p, job);
    return (int)hipGetLastError();
}

// FP64 plans: three-quarter and quarter sampling
int launch_plain_f64(const KParams &p, const KJob &job, int ws, void *stream) {
    constexpr int TQ = SHAPE_THREE_QUARTER, QS = SHAPE_QUARTER;
    if (p.shape == QS)
        return ws == 16 ? launch_plain_t<double, 16, QS>(p, job, stream) : launch_plain_t<double, 8, QS>(p, job, stream);
    return ws == 16 ? launch_plain_t<double, 16, TQ>(p, job, stream) : launch_plain_t<double, 8, TQ>(p, job, stream);
}

// FP32-state plans (three-quarter sampling only)
int launch_plain_f32(const KParams &p, const KJob &job, int ws, void *stream) {
    constexpr int TQ = SHAPE_THREE_QUARTER;
    return ws == 16 ? launch_plain_t<float, 16, TQ>(p, job, stream) : launch_plain_t<float, 8, TQ>(p, job, stream);
}

int launch_reset_counter(unsigned int *counter, void *stream) {
    reset_counter_kernel<<<dim3(1), dim3(64), 0, (hipStream_t)stream>>>(counter);
    return (int)hipGetLastError();
}

int launch_persistent_f32(const KParams &p, const KJob *d_jobs, int njobs, long long total_windows,
                          unsigned int *counter, int ws, int waves_per_block, int chunk, int grid,
                          void *stream) {
    const size_t lds = (size_t)waves_per_block * lds_bytes_per_wave(ws, false);
    if (ws == 16)
        persistent_kernel<float, 16><<<dim3(grid), dim3(64 * waves_per_block), lds, (hipStream_t)stream>>>(
            p, d_jobs, njobs, total_windows, counter, chunk);
    else
        persistent_kernel<float, 8><<<dim3(grid), dim3(64 * waves_per_block), lds, (hipStream_t)stream>>>(
            p, d_jobs, njobs, total_windows, counter, chunk);
    return (int)hipGetLastError();
}

int persistent_blocks_per_cu(int ws, int waves_per_block, int *blocks) {
    const size_t lds = (size_t)waves_per_block * lds_bytes_per_wave(ws, false);
    hipError_t e;
    if (ws == 16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, persistent_kernel<float, 16>,
                                                         64 * waves_per_block, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, persistent_kernel<float, 8>,
                                                         64 * waves_per_block, lds);
    return (int)e;
}

}  // namespace ljsde
