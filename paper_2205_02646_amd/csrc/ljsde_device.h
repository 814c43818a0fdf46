// Device helpers shared by the HIP translation units of the RL-JSDE library.
#pragma once

#include <hip/hip_runtime.h>

namespace ljsde {

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
// every source lane is valid, so no lane keeps its old value).
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Top-two of unsigned keys over the wavefront. On return every lane holds
// the largest key in `best` and the second largest in `second` (the second
// may equal the first when two lanes hold equal keys).
__device__ __forceinline__ void wave_top2_u32(unsigned &best, unsigned &second) {
    unsigned b = best, s = second, bo, so;
#define LJSDE_TOP2_STEP(CTRL)                     \
    bo = dpp_u32<CTRL>(b);                        \
    so = dpp_u32<CTRL>(s);                        \
    s = max(max(s, so), min(b, bo));              \
    b = max(b, bo);
    LJSDE_TOP2_STEP(DPP_QUAD_XOR1)
    LJSDE_TOP2_STEP(DPP_QUAD_XOR2)
    LJSDE_TOP2_STEP(DPP_ROW_HALF_MIRROR)
    LJSDE_TOP2_STEP(DPP_ROW_MIRROR)
#undef LJSDE_TOP2_STEP
    // four rows: combine their (best, second) pairs with scalar operations
    const unsigned b0 = __builtin_amdgcn_readlane(b, 0), b1 = __builtin_amdgcn_readlane(b, 16);
    const unsigned b2 = __builtin_amdgcn_readlane(b, 32), b3 = __builtin_amdgcn_readlane(b, 48);
    const unsigned s0 = __builtin_amdgcn_readlane(s, 0), s1 = __builtin_amdgcn_readlane(s, 16);
    const unsigned s2 = __builtin_amdgcn_readlane(s, 32), s3 = __builtin_amdgcn_readlane(s, 48);
    const unsigned m01 = max(b0, b1), n01 = min(b0, b1), m23 = max(b2, b3), n23 = min(b2, b3);
    best = max(m01, m23);
    second = max(max(max(s0, s1), max(s2, s3)), max(min(m01, m23), max(n01, n23)));
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
template <typename XT>
__device__ __forceinline__ void dft16_mfma(const XT *X, const signed char *Cd, const double *dft,
                                           double Pre[4][4], double Pim[4][4]) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    double x[4], gr[4], gi[4];
    int cd[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = 4 * c + q;
        x[c] = (double)X[r16 * 16 + j];
        cd[c] = Cd[r16 * 16 + j];
        const int k = (j * r16) & 15;
        gr[c] = dft[2 * k];
        gi[c] = dft[2 * k + 1];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        v4f64 tr = {0.0, 0.0, 0.0, 0.0}, ti = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double a = cd[c] == o ? x[c] : 0.0;
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

// median of three (the backend selects v_med3_u32)
__device__ __forceinline__ unsigned umed3(unsigned a, unsigned b, unsigned c) {
    return max(min(a, b), min(max(a, b), c));
}

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

}  // namespace ljsde
