// Window prologue shared by the one-window-per-wavefront kernels (plain and
// dense-C): gather the window's sensor tile, weighted by w_m of eq. (8)
// (absent pixels -> 0), its weighted energy at iteration 0, and the
// orientation-masked weighted (W/2)-point DFT P_o of eq. (12) at r = y in the
// factorised form: lane L holds the positions (L / WS + (64 / WS) t, L % WS).
#pragma once

#include "ljsde_device.h"
#include "ljsde_internal.h"

namespace ljsde {

// LDS of one wavefront: stage [NPOS][4] complex, w*y [NPOS], codes [NPOS]
template <typename T, int WS>
struct WinLds {
    static constexpr int NPOS = WS * WS;
    static constexpr size_t bytes = (size_t)NPOS * 8 * sizeof(T) + NPOS * sizeof(T) + NPOS;
};

// Returns the weighted energy E(0) (wave-reduced); fills P (QPL = WS^2 / 64
// positions x 4 orientations). `codes` are the class's per-pixel codes (-1
// outside the image). LDS of the wavefront: ldsX [NPOS] (w*y), ldsC [NPOS]
// (codes) and, for WS = 8 only (the VALU DFT), ldsS [NPOS * 8] (stage).
// WEIGHTED (general layouts): P holds P_q = DFT(w * y * A_q) for the class's
// per-pixel quadrant weights Aw [NPOS][4] instead of the code-masked spectra.
// The measurements are double or float by the job's flag (read as FP64).
template <typename T, int WS, bool WEIGHTED = false>
__device__ __forceinline__ double window_prologue(const KParams &p, const KJob &j, int bi, int bj,
                                                  const signed char *codes, T *ldsX, signed char *ldsC, T *ldsS,
                                                  C2<T> P[][4], const double *Aw = nullptr) {
    constexpr int QPL = WS * WS / 64;
    constexpr int NPOS = WS * WS;
    constexpr int KSTEP = 64 / WS;
    const int lane = threadIdx.x & 63;
    const int lam = lane % WS;
    const int krow = lane / WS;
    wave_lds_fence();  // previous window of this wave is done with the LDS

    // ---- gather the window's sensor tile (absent pixels -> 0) -------------
    const int rs = (p.B * bi - p.off) / 2;
    const int cs = (p.B * bj - p.off) / 2;
    double e0 = 0.0;
    for (int m = lane; m < NPOS; m += 64) {
        const int ip = m / WS, jp = m % WS;
        const int gi = rs + ip, gj = cs + jp;
        signed char code = codes[m];
        T x = T(0);
        if (code >= 0 && gi >= 0 && gi < j.Ms && gj >= 0 && gj < j.Ns) {
            const double yv = load_measurement(j, (size_t)gi * j.Ns + gj);
            const double wy = p.c.w[m] * yv;
            x = (T)wy;
            e0 += wy * yv;
        } else {
            code = -1;
        }
        ldsX[m] = x;
        ldsC[m] = code;
    }
    e0 = wave_sum(e0);  // weighted residual energy of eq. (8) at iteration 0
    wave_lds_fence();

    // ---- orientation-masked weighted DFT -----------------------------------
    if constexpr (WS == 16) {
        double Pre[4][4], Pim[4][4];
        if constexpr (sizeof(T) == 4 && !WEIGHTED) {
            // FP32-state plans may take the split-BF16 MFMA products (FP32
            // accumulation); ldsS (8 KiB here) is free until the spectra are staged
            if (p.dft_bf16) dft16_splitbf16<T>(ldsX, ldsC, p.c.dft, (float *)ldsS, Pre, Pim);
            else dft16_mfma<T, WEIGHTED>(ldsX, ldsC, p.c.dft, Pre, Pim, Aw);
        } else {
            dft16_mfma<T, WEIGHTED>(ldsX, ldsC, p.c.dft, Pre, Pim, Aw);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int o = 0; o < 4; ++o) P[t][o] = {(T)Pre[t][o], (T)Pim[t][o]};
    } else {
        // rows, then columns (VALU)
#pragma unroll 1
        for (int s = 0; s < QPL; ++s) {
            const int ip = krow + KSTEP * s;
            C2<T> acc[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) acc[o] = {T(0), T(0)};
#pragma unroll 2
            for (int jp = 0; jp < WS; ++jp) {
                const T x = ldsX[ip * WS + jp];
                const int c = ldsC[ip * WS + jp];
                const int k = (jp * lam) & (WS - 1);
                const T twr = (T)p.c.dft[2 * k], twi = (T)p.c.dft[2 * k + 1];
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    T xo;
                    if constexpr (WEIGHTED) xo = x * (T)Aw[(ip * WS + jp) * 4 + o];
                    else xo = (c == o) ? x : T(0);
                    acc[o].re += xo * twr;
                    acc[o].im += xo * twi;
                }
            }
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                // stage order [o][ip][l]: consecutive lanes touch consecutive entries
                ldsS[((o * WS + ip) * WS + lam) * 2] = acc[o].re;
                ldsS[((o * WS + ip) * WS + lam) * 2 + 1] = acc[o].im;
            }
        }
        wave_lds_fence();
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
            const int kap = krow + KSTEP * t;
#pragma unroll
            for (int o = 0; o < 4; ++o) P[t][o] = {T(0), T(0)};
#pragma unroll 2
            for (int ip = 0; ip < WS; ++ip) {
                const int k = (ip * kap) & (WS - 1);
                const T twr = (T)p.c.dft[2 * k], twi = (T)p.c.dft[2 * k + 1];
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    const T ar = ldsS[((o * WS + ip) * WS + lam) * 2];
                    const T ai = ldsS[((o * WS + ip) * WS + lam) * 2 + 1];
                    P[t][o].re += ar * twr - ai * twi;
                    P[t][o].im += ar * twi + ai * twr;
                }
            }
        }
    }
    wave_lds_fence();

    return e0;
}

}  // namespace ljsde
