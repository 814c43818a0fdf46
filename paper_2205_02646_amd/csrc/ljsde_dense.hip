// RL-JSDE in its dense form (Sec. IV, eqs. (11)-(18)) on gfx950.
//
// Per class (local measurement matrix), the full W^2 x W^2 matrix C of
// eq. (14) sits in device memory, FP64. A window keeps the projected residual
// R(sigma, rho) of all W^2 frequencies as its state (eq. (12) at r = y); every
// iteration selects by eq. (11), steps by eqs. (15)-(16) and subtracts
// gamma * delta times column (u, v) of C (eq. (17)). Per window-iteration the
// work is one metric per frequency, the selection and one complex
// multiply-add per frequency, and the column read is W^2 * 16 bytes (16 KiB
// at W = 32), which depends on the pick: the loop is bound by the VALU and
// the latency of that read (columns are mostly served from L2).
//
// C is built on the device from the class tables: for pixel shapes from the
// factorised form C(f, g) = sum_o conj(H_o(f)) H_o(g) S_o(f - g) (the same
// matrix as eq. (14), see ljsde_kernels.hip), for general layouts from the
// ten spectra S_qq'. It is stored so that a wavefront's read of one column
// is 16 loads of 64 consecutive complex values.
#include <hip/hip_runtime.h>

#include "ljsde_device.h"
#include "ljsde_internal.h"
#include "ljsde_window.h"

namespace ljsde {

// Frequency sigma * W + rho of entry (t, c) of lane L: position
// (k, l) = (L / WS + (64 / WS) t, L % WS), c = 2a + b for (k + WS a, l + WS b).
template <int WS>
__device__ __forceinline__ int dense_freq(int L, int t, int c) {
    constexpr int W = 2 * WS, KSTEP = 64 / WS;
    return (L / WS + KSTEP * t + WS * (c >> 1)) * W + L % WS + WS * (c & 1);
}

// Column g of C for every class of a size set: out[(cls * W^2 + g) * W^2 + e]
// with e = (4 t + c) * 64 + L the lane-ordered entry of frequency
// dense_freq(L, t, c). Grid (W^2 columns, classes), 256 threads.
template <int WS>
__global__ __launch_bounds__(256) void dense_c_build_kernel(KParams p, const unsigned char *tables, double2 *out) {
    constexpr int W = 2 * WS, NF = W * W;
    const int g = blockIdx.x;
    const int cls = blockIdx.y;
    const double *S = (const double *)(tables + (size_t)cls * p.lay.stride + p.lay.offS);
    const double *H = p.c.H;
    const int kg = (g / W) & (WS - 1), lg = (g % W) & (WS - 1);
    double Hgr[4], Hgi[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        Hgr[o] = H[((size_t)g * 4 + o) * 2];
        Hgi[o] = H[((size_t)g * 4 + o) * 2 + 1];
    }
    double2 *col = out + ((size_t)cls * NF + g) * NF;
    for (int e = threadIdx.x; e < NF; e += blockDim.x) {
        const int L = e & 63, tc = e >> 6;
        const int f = dense_freq<WS>(L, tc >> 2, tc & 3);
        const int kf = (f / W) & (WS - 1), lf = (f % W) & (WS - 1);
        const int pos = ((kf - kg) & (WS - 1)) * WS + ((lf - lg) & (WS - 1));
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const double hr = H[((size_t)f * 4 + o) * 2], hi = H[((size_t)f * 4 + o) * 2 + 1];
            // conj(H_o(f)) H_o(g)
            const double ar = hr * Hgr[o] + hi * Hgi[o], ai = hr * Hgi[o] - hi * Hgr[o];
            const double sr = S[(pos * 4 + o) * 2], si = S[(pos * 4 + o) * 2 + 1];
            re += ar * sr - ai * si;
            im += ar * si + ai * sr;
        }
        col[e] = make_double2(re, im);
    }
}

// Index of the spectrum S_qq' (q <= q') in the general-layout class tables:
// (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).
__device__ __forceinline__ int pair_index(int q, int r) {
    const int a = q < r ? q : r, b = q < r ? r : q;
    return 4 * a - (a * (a - 1)) / 2 + (b - a);
}

// Column g of C for a general layout (per-pixel quadrant weights A_m(q)):
// with a_m(f) = exp(i theta 2 (i' sigma + j' rho)) sum_q A_m(q) e_q(f) and
// e_q(f) = exp(i theta (qa sigma + qb rho)),
//     C(f, g) = sum_{q, q'} conj(e_q(f)) e_q'(g) S_qq'(f - g),
// S_qq'(k, l) = sum_m w_m A_m(q) A_m(q') exp(-2 pi i (i' k + j' l) / Ws).
// Same output order and grid as dense_c_build_kernel.
template <int WS>
__global__ __launch_bounds__(256) void dense_c_build_general_kernel(KParams p, const unsigned char *tables,
                                                                    double2 *out) {
    constexpr int W = 2 * WS, NF = W * W;
    const int g = blockIdx.x;
    const int cls = blockIdx.y;
    const double *S = (const double *)(tables + (size_t)cls * p.lay.stride + p.lay.offS);
    const double *ew = p.c.ew;
    const int sg = g / W, rg = g % W;
    const int kg = sg & (WS - 1), lg = rg & (WS - 1);
    double egr[4], egi[4];  // e_q'(g)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ph = ((q >> 1) * sg + (q & 1) * rg) & (W - 1);
        egr[q] = ew[2 * ph];
        egi[q] = ew[2 * ph + 1];
    }
    double2 *col = out + ((size_t)cls * NF + g) * NF;
    for (int e = threadIdx.x; e < NF; e += blockDim.x) {
        const int L = e & 63, tc = e >> 6;
        const int f = dense_freq<WS>(L, tc >> 2, tc & 3);
        const int sf = f / W, rf = f % W;
        const int pos = ((sf - kg) & (WS - 1)) * WS + ((rf - lg) & (WS - 1));
        const double *Sp = S + (size_t)pos * 20;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double tr = 0.0, ti = 0.0;  // sum_q' e_q'(g) S_qq'
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = pair_index(q, r);
                const double sr = Sp[2 * k], si = Sp[2 * k + 1];
                tr += egr[r] * sr - egi[r] * si;
                ti += egr[r] * si + egi[r] * sr;
            }
            const int ph = ((q >> 1) * sf + (q & 1) * rf) & (W - 1);
            const double cr = ew[2 * ph], ci = -ew[2 * ph + 1];  // conj(e_q(f))
            re += cr * tr - ci * ti;
            im += cr * ti + ci * tr;
        }
        col[e] = make_double2(re, im);
    }
}

// LDS of one wavefront. Prologue: w*y [NPOS] FP64, codes [NPOS], and the VALU
// DFT's stage [NPOS][4] complex for WS = 8 only. Loop: q / D of the class in
// lane order [W^2] FP64 (entry (4t + c) * 64 + L), over the prologue's bytes.
template <int WS>
struct DenseLds {
    static constexpr int NPOS = WS * WS;
    static constexpr size_t stage = WS == 16 ? 0 : (size_t)NPOS * 8 * 8;
    static constexpr size_t prologue = stage + (size_t)NPOS * 8 + NPOS;
    static constexpr size_t qd = (size_t)4 * WS * WS * 8;
    static constexpr size_t bytes = prologue > qd ? prologue : qd;
};

// One wavefront per window. SHAPE is a pixel-shape mask or SHAPE_GENERAL
// (per-pixel quadrant weights: P_q of every quadrant, R = sum_q conj(e_q) P_q).
// IO is the element type of the output (FP32 plans: float; the arithmetic is
// FP64 either way); the measurements are double or float by the job's flag.
// HALVES = 2 reads the column of eq. (17) in two halves through the same
// registers (the second after the first half's update): 4 wavefronts per
// SIMD instead of 3, at the price of a second exposed load latency.
template <int WS, int SHAPE, typename IO, int HALVES>
__device__ __forceinline__ void dense_window(const KParams &p, const KJob &j, const double2 *__restrict__ Cd, int wo,
                                             char *lds) {
    constexpr int W = 2 * WS, NF = W * W, NPOS = WS * WS, QPL = NPOS / 64, KSTEP = 64 / WS;
    const long long w = wo;
    const int bi = (int)(w / j.nbj), bj = (int)(w % j.nbj);
    const int lane = threadIdx.x & 63;
    const int lam = lane % WS, krow = lane / WS;

    const int cls = __builtin_amdgcn_readfirstlane(j.rowcls[bi] * j.ncolk + j.colcls[bj]);
    const unsigned char *tb = j.tables + (size_t)cls * p.lay.stride;
    const double *qD64 = (const double *)(tb + p.lay.offQD64);
    const double *invD = (const double *)(tb + p.lay.offInvD);
    const signed char *codes = (const signed char *)(tb + p.lay.offCodes);

    using LL = DenseLds<WS>;
    double *ldsS = (double *)lds;
    double *ldsX = (double *)(lds + LL::stage);
    signed char *ldsC = (signed char *)(lds + LL::stage + (size_t)NPOS * 8);
    C2<double> P[QPL][4];
    constexpr bool GENERAL = SHAPE == SHAPE_GENERAL;
    constexpr int PSHAPE = GENERAL ? SHAPE_QUARTER : SHAPE;  // Q_q = P_q
    const double *Aw = GENERAL ? (const double *)(tb + p.lay.offA) : nullptr;
    const double e0 = window_prologue<double, WS, GENERAL>(p, j, bi, bj, codes, ldsX, ldsC, ldsS, P, Aw);

    // R(0) of eq. (12) through the factorised projection, and q / D
    const double *ew = p.c.ew;
    const C2<double> tl = {ew[2 * lam], -ew[2 * lam + 1]};
    C2<double> R[QPL][4];
    double *ldsQ = (double *)lds;  // after the prologue
#pragma unroll
    for (int t = 0; t < QPL; ++t) {
        const int kap = krow + KSTEP * t;
        const C2<double> tk = {ew[2 * kap], -ew[2 * kap + 1]};
        const C2<double> tkl = {ew[2 * (kap + lam)], -ew[2 * (kap + lam) + 1]};
        project4<double, PSHAPE>(P[t], tl, tk, tkl, R[t]);
#pragma unroll
        for (int c = 0; c < 4; ++c) ldsQ[(4 * t + c) * 64 + lane] = qD64[dense_freq<WS>(lane, t, c)];
    }

    const double2 *Cc = Cd + (size_t)cls * NF * NF;
    const int BB = p.B * p.B;
    const int oi = lane / p.B, oj = lane % p.B;
    double outacc = 0.0;
    double E = e0;
    int nu_done = 0;

#pragma unroll 1
    for (int nu = 0; nu < p.iters; ++nu) {
        // eq. (11): q |R|^2 / D. The first maximum in sigma * W + rho order,
        // ties within TIE_REL included: the lowest index whose metric reaches
        // M (1 - TIE_REL), M the wavefront maximum. Within a lane the index
        // grows with (a, t, b) for c = 2a + b.
        int lq = lane;
        asm volatile("" : "+v"(lq));  // q / D is re-read from LDS every iteration, not held in registers
        double m[QPL][4];
#pragma unroll
        for (int t = 0; t < QPL; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                m[t][c] = (R[t][c].re * R[t][c].re + R[t][c].im * R[t][c].im) * ldsQ[(4 * t + c) * 64 + lq];
        // Fast path: a key per frequency from the upper word of its FP64
        // metric (sign, exponent, 20 mantissa bits; the lowest 4 replaced by
        // the frequency's in-lane code 4t + c), the lane's largest and
        // second-largest key and the wavefront maximum. The keys keep the
        // metric to 2^-16 relative, so when exactly one key reaches (1 - 1e-4)
        // of the maximum, its frequency is the FP64 maximum and no other
        // metric lies within TIE_REL of it: the tie rule would pick the same.
        // Otherwise (ties, near ties, all metrics zero) the exact rule decides.
        int idx;
        {
            unsigned kb = 0u, ks = 0u;
#pragma unroll
            for (int t = 0; t < QPL; ++t) {
                unsigned key[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    key[c] = ((unsigned)__double2hiint(m[t][c]) & ~15u) | (unsigned)(4 * t + c);
                ks = max(ks, umed3(kb, key[0], key[1]));
                kb = umax3(kb, key[0], key[1]);
                ks = max(ks, umed3(kb, key[2], key[3]));
                kb = umax3(kb, key[2], key[3]);
            }
            const unsigned M = wave_max_u32(kb);
            const unsigned thr = (unsigned)__double2hiint(__hiloint2double((int)(M & ~15u), 0) * (1.0 - 1e-4));
            const unsigned long long hi1 = __ballot(kb >= thr);
            const unsigned long long hi2 = __ballot(ks >= thr);
            if (__popcll(hi1) == 1 && hi2 == 0ull) {
                const int L = __builtin_ctzll(hi1);
                const int code = (int)(M & 15u);
                const int t = code >> 2, a = (code >> 1) & 1, b = code & 1;
                idx = ((L / WS) + KSTEP * t + WS * a) * W + (L % WS) + WS * b;
            } else {
                idx = select_lowest_max<double, WS, QPL>(m, TIE_REL, lane);
            }
        }
        const int u = idx / W, v = idx % W;

        // eq. (17) needs column (u, v) of C: start its loads now
        const double2 *col = Cc + (size_t)idx * NF + lane;
        constexpr int TH = QPL / HALVES > 0 ? QPL / HALVES : 1;  // positions per half
        double2 cv[TH][4];
#pragma unroll
        for (int t = 0; t < TH; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) cv[t][c] = col[(4 * t + c) * 64];
        const double id = invD[idx];

        // R_uv from its owner lane (uniform branch on the owner's register)
        const int ku = u % WS, lv = v % WS;
        const int code = 4 * (ku / KSTEP) + 2 * (u / WS) + v / WS;
        const int owner = (ku % KSTEP) * WS + lv;
        double rr = 0.0, ri = 0.0;
#pragma unroll
        for (int t = 0; t < QPL; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (code == 4 * t + c) {
                    rr = readlane_f64(R[t][c].re, owner);
                    ri = readlane_f64(R[t][c].im, owner);
                }

        // eqs. (15)-(16) and the energy of eq. (8)
        const double gr = p.gamma * rr * id, gi = p.gamma * ri * id;
        E = uniform_f64(E - p.ecoef * (rr * rr + ri * ri) * id);
        // eq. (18) on the central block, pick by pick
        if (lane < BB) {
            const int ph = ((p.off + oi) * u + (p.off + oj) * v) & (W - 1);
            outacc += gr * ew[2 * ph] - gi * ew[2 * ph + 1];
        }
        if (j.sel != nullptr && lane == 0) j.sel[w * p.iters + nu] = (int16_t)idx;
        nu_done = nu + 1;
        if (p.tau > 0.0 && E <= p.tau * e0) break;

        // eq. (17): R -= gamma delta C(:, (u, v))
#pragma unroll
        for (int h = 0; h * TH < QPL; ++h) {
            if (h > 0) {
#pragma unroll
                for (int t = 0; t < TH; ++t)
#pragma unroll
                    for (int c = 0; c < 4; ++c) cv[t][c] = col[(4 * (h * TH + t) + c) * 64];
            }
#pragma unroll
            for (int t = 0; t < TH; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) {  // two fused multiply-adds per component
                    C2<double> &r = R[h * TH + t][c];
                    r.re = fma(-gr, cv[t][c].x, fma(gi, cv[t][c].y, r.re));
                    r.im = fma(-gr, cv[t][c].y, fma(-gi, cv[t][c].x, r.im));
                }
        }
    }
    if (j.sel != nullptr)
        for (int nu = nu_done + lane; nu < p.iters; nu += 64) j.sel[w * p.iters + nu] = -1;
    if (lane < BB) {
        IO *O = (IO *)j.out;
        const size_t row = (size_t)(p.B * bi + oi);
        O[row * (size_t)(2 * j.Ns) + (size_t)(p.B * bj + oj)] = (IO)outacc;
    }
}

// One image: workgroup b runs window order[b] (class-sorted, per-XCD chunks).
template <int WS, int SHAPE, typename IO, int HALVES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HALVES == 2 ? 4 : 3))) void dense_kernel(
    KParams p, KJob j, const double2 *__restrict__ Cd, const int *__restrict__ order) {
    extern __shared__ __align__(16) char lds[];
    const int wo = order[blockIdx.x];
    if (wo < 0) return;
    dense_window<WS, SHAPE, IO, HALVES>(p, j, Cd, wo, lds);
}

// Many images in one launch: workgroup b runs window order[b].y of job
// order[b].x (x < 0: idle), with the job's own dense C.
template <int WS, int SHAPE, typename IO, int HALVES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HALVES == 2 ? 4 : 3))) void dense_batch_kernel(
    KParams p, const KJob *__restrict__ jobs, const int2 *__restrict__ order) {
    extern __shared__ __align__(16) char lds[];
    const int2 e = order[blockIdx.x];
    if (e.x < 0) return;
    const KJob J = jobs[e.x];
    dense_window<WS, SHAPE, IO, HALVES>(p, J, (const double2 *)J.dense, e.y, lds);
}

size_t dense_c_bytes(int ws, int n_classes) {
    const size_t nf = (size_t)(2 * ws) * (2 * ws);
    return (size_t)n_classes * nf * nf * sizeof(double2);
}

int launch_dense_c_build(const KParams &p, const unsigned char *tables, int n_classes, int ws, void *out,
                         void *stream) {
    if (n_classes <= 0) return 0;
    const int nf = (2 * ws) * (2 * ws);
    const dim3 grid((unsigned)nf, (unsigned)n_classes);
    hipStream_t st = (hipStream_t)stream;
    if (p.shape == SHAPE_GENERAL) {
        if (ws == 16) dense_c_build_general_kernel<16><<<grid, dim3(256), 0, st>>>(p, tables, (double2 *)out);
        else dense_c_build_general_kernel<8><<<grid, dim3(256), 0, st>>>(p, tables, (double2 *)out);
    } else {
        if (ws == 16) dense_c_build_kernel<16><<<grid, dim3(256), 0, st>>>(p, tables, (double2 *)out);
        else dense_c_build_kernel<8><<<grid, dim3(256), 0, st>>>(p, tables, (double2 *)out);
    }
    return (int)hipGetLastError();
}

template <int WS, int SHAPE, typename IO>
static int launch_dense_t(const KParams &p, const KJob &job, const void *C, const int *order, int n,
                          void *stream) {
    if (n <= 0) return 0;
    // W = 32: the column in two halves (measured 1.04x over one piece: the
    // fourth wavefront per SIMD hides more of the pick-dependent load latency
    // than the second exposed latency costs); W = 16 holds one position per lane
    constexpr int HALVES = WS == 16 ? 2 : 1;
    dense_kernel<WS, SHAPE, IO, HALVES><<<dim3((unsigned)n), dim3(64), DenseLds<WS>::bytes, (hipStream_t)stream>>>(
        p, job, (const double2 *)C, order);
    return (int)hipGetLastError();
}

template <typename IO>
static int launch_dense_io(const KParams &p, const KJob &job, const void *C, const int *order, int n, int ws,
                           void *stream) {
    constexpr int TQ = SHAPE_THREE_QUARTER, QS = SHAPE_QUARTER, GN = SHAPE_GENERAL;
    if (p.shape == GN)
        return ws == 16 ? launch_dense_t<16, GN, IO>(p, job, C, order, n, stream)
                        : launch_dense_t<8, GN, IO>(p, job, C, order, n, stream);
    if (p.shape == QS)
        return ws == 16 ? launch_dense_t<16, QS, IO>(p, job, C, order, n, stream)
                        : launch_dense_t<8, QS, IO>(p, job, C, order, n, stream);
    return ws == 16 ? launch_dense_t<16, TQ, IO>(p, job, C, order, n, stream)
                    : launch_dense_t<8, TQ, IO>(p, job, C, order, n, stream);
}

template <int WS, int SHAPE, typename IO>
static int launch_dense_batch_t(const KParams &p, const KJob *jobs, const void *order, int n, void *stream) {
    if (n <= 0) return 0;
    constexpr int HALVES = WS == 16 ? 2 : 1;
    dense_batch_kernel<WS, SHAPE, IO, HALVES>
        <<<dim3((unsigned)n), dim3(64), DenseLds<WS>::bytes, (hipStream_t)stream>>>(p, jobs, (const int2 *)order);
    return (int)hipGetLastError();
}

template <typename IO>
static int launch_dense_batch_io(const KParams &p, const KJob *jobs, const void *order, int n, int ws,
                                 void *stream) {
    constexpr int TQ = SHAPE_THREE_QUARTER, QS = SHAPE_QUARTER, GN = SHAPE_GENERAL;
    if (p.shape == GN)
        return ws == 16 ? launch_dense_batch_t<16, GN, IO>(p, jobs, order, n, stream)
                        : launch_dense_batch_t<8, GN, IO>(p, jobs, order, n, stream);
    if (p.shape == QS)
        return ws == 16 ? launch_dense_batch_t<16, QS, IO>(p, jobs, order, n, stream)
                        : launch_dense_batch_t<8, QS, IO>(p, jobs, order, n, stream);
    return ws == 16 ? launch_dense_batch_t<16, TQ, IO>(p, jobs, order, n, stream)
                    : launch_dense_batch_t<8, TQ, IO>(p, jobs, order, n, stream);
}

int launch_dense_batch(const KParams &p, const KJob *jobs, const void *order, int n, int ws, bool f32io,
                       void *stream) {
    return f32io ? launch_dense_batch_io<float>(p, jobs, order, n, ws, stream)
                 : launch_dense_batch_io<double>(p, jobs, order, n, ws, stream);
}

int launch_dense(const KParams &p, const KJob &job, const void *C, const int *order, int n, int ws, bool f32io,
                 void *stream) {
    return f32io ? launch_dense_io<float>(p, job, C, order, n, ws, stream)
                 : launch_dense_io<double>(p, job, C, order, n, ws, stream);
}

}  // namespace ljsde
