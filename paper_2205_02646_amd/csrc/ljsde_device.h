// Device helpers shared by the HIP translation units of the RL-JSDE library.
#pragma once

#include <hip/hip_runtime.h>

#include "ljsde_internal.h"

namespace ljsde {

// Measurement i of a job (row-major), widened to FP64: double or float
// storage by the job's wave-uniform flag.
__device__ __forceinline__ double load_measurement(const KJob &j, size_t i) {
    return j.y64 ? ((const double *)j.y)[i] : (double)((const float *)j.y)[i];
}

template <typename T>
struct C2 {
    T re, im;
};

// Orders this wavefront's LDS accesses across lanes (a single wave needs no
// barrier, only a wait for its own LDS operations).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// DPP lane move inside rows of 16 lanes (quad_perm / mirror controls only:
// every source lane is valid). The fill value 0 is the identity of an
// unsigned max, which lets the move fold into a v_max_u32 with a DPP operand.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Pixel shapes (Sec. I; Sec. II eq. (1)): a pixel of code o collects light on
// the quadrants o ^ d for the bits d of a 4-bit mask. Three-quarter sampling
// (every quadrant but the opaque one, o) is 0xE; quarter sampling (only the
// transparent quadrant, o) is 0x1.
constexpr int SHAPE_THREE_QUARTER = 0xE;
constexpr int SHAPE_QUARTER = 0x1;

// Per-quadrant sums of the projection. With H_o = sum_{d in mask} e_{o ^ d}
// (e_q the response of quadrant q), sum_o conj(H_o) P_o = sum_q conj(e_q) Q_q
// where Q_q = sum_{d in mask} P_{q ^ d}.
template <int MASK, typename T>
__device__ __forceinline__ void shape_sums(const C2<T> P[4], C2<T> Q[4]) {
    if constexpr (MASK == SHAPE_THREE_QUARTER) {
        const C2<T> sp = {P[0].re + P[1].re + P[2].re + P[3].re, P[0].im + P[1].im + P[2].im + P[3].im};
#pragma unroll
        for (int q = 0; q < 4; ++q) Q[q] = {sp.re - P[q].re, sp.im - P[q].im};
    } else if constexpr (MASK == SHAPE_QUARTER) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Q[q] = P[q];
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Q[q] = {T(0), T(0)};
#pragma unroll
            for (int d = 0; d < 4; ++d)
                if ((MASK >> d) & 1) Q[q] = {Q[q].re + P[q ^ d].re, Q[q].im + P[q ^ d].im};
        }
    }
}

// R(a, b) for the four frequencies (k + Ws a, l + Ws b) of one position:
// R = sum_q (-1)^(qa a + qb b) e^{-i theta (qa k + qb l)} Q_q, with the
// per-quadrant sums Q_q of the pixel shape (sum_o P_o - P_q for the L pixels
// of three-quarter sampling).
template <typename T, int SHAPE>
__device__ __forceinline__ void project4(const C2<T> P[4], C2<T> tl, C2<T> tk, C2<T> tkl, C2<T> R[4]) {
    C2<T> Q[4];
    shape_sums<SHAPE, T>(P, Q);
    const C2<T> q0 = Q[0], q1 = Q[1], q2 = Q[2], q3 = Q[3];
    const C2<T> u1 = {tl.re * q1.re - tl.im * q1.im, tl.re * q1.im + tl.im * q1.re};
    const C2<T> u2 = {tk.re * q2.re - tk.im * q2.im, tk.re * q2.im + tk.im * q2.re};
    const C2<T> u3 = {tkl.re * q3.re - tkl.im * q3.im, tkl.re * q3.im + tkl.im * q3.re};
    const C2<T> s1 = {q0.re + u3.re, q0.im + u3.im}, d1 = {q0.re - u3.re, q0.im - u3.im};
    const C2<T> s2 = {u1.re + u2.re, u1.im + u2.im}, d2 = {u1.re - u2.re, u1.im - u2.im};
    R[0] = {s1.re + s2.re, s1.im + s2.im};  // (a, b) = (0, 0)
    R[1] = {d1.re - d2.re, d1.im - d2.im};  // (0, 1)
    R[2] = {d1.re + d2.re, d1.im + d2.im};  // (1, 0)
    R[3] = {s1.re - s2.re, s1.im - s2.im};  // (1, 1)
}

// Maximum of unsigned keys over the wavefront (a wave-uniform value): a
// max-butterfly inside each row of 16 lanes, then the four row maxima.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, dpp_u32<DPP_QUAD_XOR1>(v));
    v = max(v, dpp_u32<DPP_QUAD_XOR2>(v));
    v = max(v, dpp_u32<DPP_ROW_HALF_MIRROR>(v));
    v = max(v, dpp_u32<DPP_ROW_MIRROR>(v));
    const unsigned r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const unsigned r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    // the four row maxima are scalars: reduce them on the scalar unit (left
    // to itself the compiler forms a vector max3 and copies two of them into
    // vector registers for it)
    unsigned m01, m23, m;
    asm("s_max_u32 %0, %1, %2" : "=s"(m01) : "s"(r0), "s"(r1));
    asm("s_max_u32 %0, %1, %2" : "=s"(m23) : "s"(r2), "s"(r3));
    asm("s_max_u32 %0, %1, %2" : "=s"(m) : "s"(m01), "s"(m23));
    return m;
}

// Selection ties (eqs. (10)-(11)): metrics within a relative TIE_REL of the
// maximum count as maximal, and the lowest frequency index sigma * W + rho
// among them wins. Streaming form for candidates visited in increasing index
// order, and the merge of two partial results.
constexpr double TIE_REL = 1e-10;

template <typename T>
__device__ __forceinline__ void tie_keep(T &best, int &code, T m, int c, T eps) {
    if (m > best * (T(1) + eps)) {
        best = m;
        code = c;
    } else if (m > best) {
        best = m;  // inside the tie band: the earlier (lower) index stays
    }
}

template <typename T>
__device__ __forceinline__ void tie_merge(T &best, int &idx, T ob, int oi, T eps) {
    if (ob > best * (T(1) + eps)) {
        best = ob;
        idx = oi;
    } else if (!(best > ob * (T(1) + eps))) {
        best = best > ob ? best : ob;
        idx = idx < oi ? idx : oi;
    }
}

typedef double v4f64 __attribute__((ext_vector_type(4)));

// Orientation-masked 16-point 2-D DFT of one window on FP64 MFMA
// (v_mfma_f64_16x16x4f64), for all four orientations:
//     P_o(k, l) = sum_{i, j} X(i, j) [code(i, j) = o] e^{-2 pi i (i k + j l) / 16}
// as T = X_o G, P_o = G T with G(a, b) = e^{-2 pi i a b / 16} (symmetric).
// MFMA 16x16x4 operands: lane L supplies A[L % 16][4c + L / 16] and
// B[4c + L / 16][L % 16] for K-chunk c; the result holds D[L / 16 + 4r][L % 16]
// in register r. The first product therefore leaves in register c exactly the
// B operand the second one needs for chunk c, and the second leaves lane L
// with P_o(L / 16 + 4t, L % 16) in register t: the positions this lane owns.
// X is w * y in LDS ([i][j], absent pixels 0), Cd the codes, dft the table of
// e^{-2 pi i k / 16}. Needs the whole wavefront active.
// WEIGHTED: general per-pixel quadrant weights instead of codes,
//     P_q(k, l) = sum_{i, j} X(i, j) A(i, j, q) e^{-2 pi i (i k + j l) / 16}
// with Aw = A as [i * 16 + j][q] (Cd unused).
template <typename XT, bool WEIGHTED = false>
__device__ __forceinline__ void dft16_mfma(const XT *X, const signed char *Cd, const double *dft,
                                           double Pre[4][4], double Pim[4][4], const double *Aw = nullptr) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // per call: lane-derived addresses are not hoisted into registers
    const int r16 = lane & 15, q = lane >> 4;
    double x[4], gr[4], gi[4];
    int cd[4];
    double aw[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = 4 * c + q;
        x[c] = (double)X[r16 * 16 + j];
        if constexpr (WEIGHTED) {
#pragma unroll
            for (int o = 0; o < 4; ++o) aw[c][o] = Aw[(r16 * 16 + j) * 4 + o];
        } else {
            cd[c] = Cd[r16 * 16 + j];
        }
        const int k = (j * r16) & 15;
        gr[c] = dft[2 * k];
        gi[c] = dft[2 * k + 1];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        v4f64 tr = {0.0, 0.0, 0.0, 0.0}, ti = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double a;
            if constexpr (WEIGHTED) a = x[c] * aw[c][o];
            else a = cd[c] == o ? x[c] : 0.0;
            tr = __builtin_amdgcn_mfma_f64_16x16x4f64(a, gr[c], tr, 0, 0, 0);
            ti = __builtin_amdgcn_mfma_f64_16x16x4f64(a, gi[c], ti, 0, 0, 0);
        }
        v4f64 pr = {0.0, 0.0, 0.0, 0.0}, pi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            pr = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[c], tr[c], pr, 0, 0, 0);
            pr = __builtin_amdgcn_mfma_f64_16x16x4f64(-gi[c], ti[c], pr, 0, 0, 0);
            pi = __builtin_amdgcn_mfma_f64_16x16x4f64(gr[c], ti[c], pi, 0, 0, 0);
            pi = __builtin_amdgcn_mfma_f64_16x16x4f64(gi[c], tr[c], pi, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            Pre[t][o] = pr[t];
            Pim[t][o] = pi[t];
        }
    }
}

typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// Same DFT as dft16_mfma with 3-term split-BF16 products on
// v_mfma_f32_16x16x32_bf16 and FP32 accumulation: x = x_h + x_l with
// x_h = bf16(x), x_l = bf16(x - x_h), and x g ~ x_h g_h + x_l g_h + x_h g_l.
// The K = 32 of the instruction holds two 16-terms: [X_h | X_l] [G_h; G_h]
// gives X_h G_h + X_l G_h, [X_h | X_l] [G_l; 0] gives X_h G_l. Operands: lane L
// supplies A[L % 16][8 (L / 16) + e] and B[8 (L / 16) + e][L % 16] (e < 8); the
// result holds D[4 (L / 16) + r][L % 16], so the intermediate and the result
// pass through `lds` (>= 2 x 256 floats, wavefront-private) to reach the
// layout of the next step. Relative error ~2^-16.
template <typename XT>
__device__ __forceinline__ void dft16_splitbf16(const XT *X, const signed char *Cd, const double *dft,
                                                float *lds, double Pre[4][4], double Pim[4][4]) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // per call: lane-derived addresses are not hoisted into registers
    const int r16 = lane & 15, q = lane >> 4;
    const bool low = q >= 2;           // this lane feeds the second 16 of K
    const int k0 = 8 * (q & 1);        // first row/column (mod 16) of its 8 elements
    // G(k0 + e, r16) = G(r16, k0 + e): the B operand of the first product and
    // the A operand of the second are the same values
    v8bf16 GrHH, GrL0, GiHH, GiL0, nGiHH, nGiL0;
    float xv[8];
    int cd[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = ((k0 + e) * r16) & 15;
        const float gr = (float)dft[2 * k], gi = (float)dft[2 * k + 1];
        const __bf16 grh = (__bf16)gr, gih = (__bf16)gi;
        const __bf16 grl = (__bf16)(gr - (float)grh), gil = (__bf16)(gi - (float)gih);
        GrHH[e] = grh;
        GiHH[e] = gih;
        nGiHH[e] = (__bf16)(-(float)gih);
        GrL0[e] = low ? (__bf16)0.0f : grl;
        GiL0[e] = low ? (__bf16)0.0f : gil;
        nGiL0[e] = low ? (__bf16)0.0f : (__bf16)(-(float)gil);
        xv[e] = (float)X[r16 * 16 + k0 + e];
        cd[e] = Cd[r16 * 16 + k0 + e];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        v8bf16 A1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = cd[e] == o ? xv[e] : 0.0f;
            const __bf16 h = (__bf16)x;
            A1[e] = low ? (__bf16)(x - (float)h) : h;
        }
        v4f32 tr = {0.f, 0.f, 0.f, 0.f}, ti = {0.f, 0.f, 0.f, 0.f};
        tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, GrHH, tr, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, GrL0, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, GiHH, ti, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, GiL0, ti, 0, 0, 0);
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // T[4q + r][r16], real plane then imaginary plane
            lds[(4 * q + r) * 16 + r16] = tr[r];
            lds[256 + (4 * q + r) * 16 + r16] = ti[r];
        }
        wave_lds_fence();
        v8bf16 BTr, BTi;  // [T_h; T_l]
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float a = lds[(k0 + e) * 16 + r16], b = lds[256 + (k0 + e) * 16 + r16];
            const __bf16 ah = (__bf16)a, bh = (__bf16)b;
            BTr[e] = low ? (__bf16)(a - (float)ah) : ah;
            BTi[e] = low ? (__bf16)(b - (float)bh) : bh;
        }
        v4f32 pr = {0.f, 0.f, 0.f, 0.f}, pi = {0.f, 0.f, 0.f, 0.f};
        pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GrHH, BTr, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GrL0, BTr, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nGiHH, BTi, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nGiL0, BTi, pr, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GrHH, BTi, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GrL0, BTi, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GiHH, BTr, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(GiL0, BTr, pi, 0, 0, 0);
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // P[4q + r][r16]
            lds[(4 * q + r) * 16 + r16] = pr[r];
            lds[256 + (4 * q + r) * 16 + r16] = pi[r];
        }
        wave_lds_fence();
#pragma unroll
        for (int t = 0; t < 4; ++t) {  // this lane's positions (q + 4t, r16)
            Pre[t][o] = (double)lds[(q + 4 * t) * 16 + r16];
            Pim[t][o] = (double)lds[256 + (q + 4 * t) * 16 + r16];
        }
    }
    wave_lds_fence();
}

// median of three (the backend selects v_med3_u32)
__device__ __forceinline__ unsigned umed3(unsigned a, unsigned b, unsigned c) {
    return max(min(a, b), min(max(a, b), c));
}

__device__ __forceinline__ unsigned umax3(unsigned a, unsigned b, unsigned c) { return max(max(a, b), c); }

__device__ __forceinline__ double uniform_f64(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// DPP lane move of a 64-bit value inside rows of 16 lanes (quad_perm and
// mirror controls only: every source lane is valid).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ unsigned dpp_min_fill(unsigned v) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Wavefront maximum of a nonnegative value: within rows of 16 by DPP (quad
// xor 1, quad xor 2, half-row mirror, row mirror leave every lane with its
// row's maximum), then across the four rows. Uniform result.
__device__ __forceinline__ double wave_max_nonneg(double v) {
    v = fmax(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmax(v, dpp_f64<DPP_QUAD_XOR2>(v));
    v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR>(v));
    v = fmax(v, dpp_f64<DPP_ROW_MIRROR>(v));
    const double a = readlane_f64(v, 0), b = readlane_f64(v, 16), c = readlane_f64(v, 32), d = readlane_f64(v, 48);
    return fmax(fmax(a, b), fmax(c, d));
}

__device__ __forceinline__ float wave_max_nonneg(float v) {
    v = fmaxf(v, dpp_f32<DPP_QUAD_XOR1>(v));
    v = fmaxf(v, dpp_f32<DPP_QUAD_XOR2>(v));
    v = fmaxf(v, dpp_f32<DPP_ROW_HALF_MIRROR>(v));
    v = fmaxf(v, dpp_f32<DPP_ROW_MIRROR>(v));
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// Wavefront minimum of an unsigned value, same scheme. Uniform result.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
    v = min(v, dpp_min_fill<DPP_QUAD_XOR1>(v));
    v = min(v, dpp_min_fill<DPP_QUAD_XOR2>(v));
    v = min(v, dpp_min_fill<DPP_ROW_HALF_MIRROR>(v));
    v = min(v, dpp_min_fill<DPP_ROW_MIRROR>(v));
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}

// Selection of eqs. (10)/(11) over the metrics m[t][c] of a wavefront whose
// lane L holds the frequencies ((L / WS + (64 / WS) t + WS a) W + L % WS + WS b,
// c = 2a + b, t < QPL): the lowest index whose metric reaches M (1 - eps), M
// the wavefront maximum (eps = TIE_REL: ties within TIE_REL go to the lowest
// index; eps = 0: the first maximum). Metrics are nonnegative. Uniform result.
template <typename T, int WS, int QPL>
__device__ __forceinline__ int select_lowest_max(const T m[][4], T eps, int lane) {
    constexpr int W = 2 * WS, KSTEP = 64 / WS, N = 4 * QPL;
    // reductions as trees: short dependency chains
    T v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = m[i >> 2][i & 3];
#pragma unroll
    for (int s = 1; s < N; s *= 2)
#pragma unroll
        for (int i = 0; i + s < N; i += 2 * s) v[i] = fmax(v[i], v[i + s]);
    const T thr = wave_max_nonneg(v[0]) * (T(1) - eps);
    // rank r = 8a + 2t + b orders this lane's indices (16: none reaches thr)
    unsigned r[N];
#pragma unroll
    for (int t = 0; t < QPL; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) r[4 * t + c] = m[t][c] >= thr ? (unsigned)(8 * (c >> 1) + 2 * t + (c & 1)) : 16u;
#pragma unroll
    for (int s = 1; s < N; s *= 2)
#pragma unroll
        for (int i = 0; i + s < N; i += 2 * s) r[i] = min(r[i], r[i + s]);
    const int rank = (int)r[0];
    const int ra = rank >> 3, rt = (rank >> 1) & 3, rb = rank & 1;
    const unsigned fidx = rank == 16 ? 0xFFFFFFFFu
                                     : (unsigned)((lane / WS + KSTEP * rt + WS * ra) * W + lane % WS + WS * rb);
    return (int)wave_min_u32(fidx);
}

}  // namespace ljsde
