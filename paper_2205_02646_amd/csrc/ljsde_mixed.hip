// FP32-search RL-JSDE kernels for gfx950 with an FP64 loop state.
//
// The per-window state is the factorised projected residual P_o(k, l) (one
// (W/2)-point DFT of the weighted residual per opaque-quadrant orientation,
// see ljsde_kernels.hip). Here it is kept in FP64 and updated with FP64 FMAs
// (full rate on CDNA, like unpacked FP32), while the projection through the
// L-pixel responses, the eq. (11) metric and the argmax search run in FP32.
// Greedy selection is discontinuous: when the two best FP32 metrics of an
// iteration are closer than a relative NEAR_TIE, the iteration's selection is
// re-decided from the FP64 state in FP64 (first maximum in sigma * W + rho
// order). The step of eqs. (15)-(16), the energy of eq. (8) and the
// back-transform of eq. (18) are FP64.
//
// A workgroup holds NW wavefronts that model NW windows of the same class
// (same local measurement matrix), so the class's FP64 weighted-mask spectra
// S_o are staged in LDS once per group and shared.
#include <hip/hip_runtime.h>

#include "ljsde_device.h"
#include "ljsde_internal.h"

namespace ljsde {

constexpr float NEAR_TIE = 1e-4f;

// Constant address space view of read-only tables: wave-uniform indexing
// then compiles to scalar loads.
typedef const double __attribute__((address_space(4))) CDouble;
// Global address space view of the selection trace: its stores are then
// global (vector-memory counter only) rather than flat, whose completion also
// holds up the waits on LDS reads.
typedef int16_t __attribute__((address_space(1))) GInt16;

// R(a, b) of one position in FP32: the same linear map as project4. The
// per-quadrant sums of three-quarter sampling come from two pair sums (each
// Q_q adds the three orientations other than q: 12 operations instead of 14),
// and the twiddle products are folded into the 2 x 2 Walsh-Hadamard step as
// fused multiply-adds, the differences taken as 2 x - s:
//   s1 = Q_0 + t_kl Q_3, d1 = 2 Q_0 - s1; u1 = t_l Q_1, s2 = u1 + t_k Q_2,
//   d2 = 2 u1 - s2; R = (s1 + s2, d1 - d2, d1 + d2, s1 - s2).
// 36 operations per position instead of 40, in longer dependency chains
// (the FP32 search's error test replays exactly this order).
template <int SHAPE>
__device__ __forceinline__ void project4_f32(const C2<float> P[4], C2<float> tl, C2<float> tk, C2<float> tkl,
                                             C2<float> R[4]) {
    C2<float> Q[4];
    if constexpr (SHAPE == SHAPE_THREE_QUARTER) {
        const C2<float> a = {P[0].re + P[1].re, P[0].im + P[1].im};
        const C2<float> b = {P[2].re + P[3].re, P[2].im + P[3].im};
        Q[0] = {P[1].re + b.re, P[1].im + b.im};
        Q[1] = {P[0].re + b.re, P[0].im + b.im};
        Q[2] = {a.re + P[3].re, a.im + P[3].im};
        Q[3] = {a.re + P[2].re, a.im + P[2].im};
    } else {
        shape_sums<SHAPE, float>(P, Q);
    }
    const C2<float> s1 = {fmaf(tkl.re, Q[3].re, fmaf(-tkl.im, Q[3].im, Q[0].re)),
                          fmaf(tkl.re, Q[3].im, fmaf(tkl.im, Q[3].re, Q[0].im))};
    const C2<float> d1 = {fmaf(2.0f, Q[0].re, -s1.re), fmaf(2.0f, Q[0].im, -s1.im)};
    const C2<float> u1 = {fmaf(tl.re, Q[1].re, -tl.im * Q[1].im), fmaf(tl.re, Q[1].im, tl.im * Q[1].re)};
    const C2<float> s2 = {fmaf(tk.re, Q[2].re, fmaf(-tk.im, Q[2].im, u1.re)),
                          fmaf(tk.re, Q[2].im, fmaf(tk.im, Q[2].re, u1.im))};
    const C2<float> d2 = {fmaf(2.0f, u1.re, -s2.re), fmaf(2.0f, u1.im, -s2.im)};
    R[0] = {s1.re + s2.re, s1.im + s2.im};  // (a, b) = (0, 0)
    R[1] = {d1.re - d2.re, d1.im - d2.im};  // (0, 1)
    R[2] = {d1.re + d2.re, d1.im + d2.im};  // (1, 0)
    R[3] = {s1.re - s2.re, s1.im - s2.im};  // (1, 1)
}

template <int WS>
struct MixedLds {
    static constexpr int NPOS = WS * WS;
    static constexpr int W = 2 * WS;
    static constexpr int QPL = NPOS / 64;
    // per workgroup: S_o [4][NPOS] complex double; per-lane q/D [QPL][64][4] float and
    // projection twiddles [QPL][64][4] float; the twiddle tables; a work slot
    static constexpr size_t offQd = (size_t)NPOS * 64;
    static constexpr size_t offTw = offQd + (size_t)QPL * 64 * 16;
    static constexpr size_t offTab = offTw + (size_t)QPL * 64 * 16;
    static constexpr size_t offSlot = offTab + (size_t)(2 * WS + 2 * W) * 8;
    static constexpr size_t shared_bytes = offSlot + 64;
    // per wavefront: w*y [NPOS] double and codes [NPOS] (after the prologue:
    // the kept picks, [NPOS / 2] complex steps and [NPOS / 2] int16
    // frequencies), then, for the window DFTs that pass a stage through LDS
    // (the VALU passes, which W = 16 always takes, and the split-BF16
    // products), the stage [NPOS] complex double
    static constexpr size_t offCodes = (size_t)NPOS * 8;
    static constexpr size_t offStage = (size_t)NPOS * 9;
    static constexpr bool has_stage(bool vdft_or_bf16) { return WS != 16 || vdft_or_bf16; }
    static constexpr size_t wave_bytes(bool vdft_or_bf16) {
        return offStage + (has_stage(vdft_or_bf16) ? (size_t)NPOS * 16 : 0);
    }
    static constexpr size_t bytes(int nw, bool vdft_or_bf16) { return shared_bytes + nw * wave_bytes(vdft_or_bf16); }
};

// The lane index, derived afresh where it is used (the count of execution-mask
// bits below the lane). The asm is volatile, so nothing computed from it is
// evaluated ahead of the iteration loop and carried through it in registers
// (at four wavefronts per SIMD such values are spilled to scratch memory).
__device__ __forceinline__ int fresh_lane() {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// Launch-variant knobs of the FP32 kernels (picked by the autotuner):
//  QREG  the per-lane q/D and projection twiddles of the window's class are
//        loaded from LDS into registers once per window (more VGPRs, fewer
//        LDS reads) instead of being re-read from LDS every iteration;
//  VDFT  the window DFT runs as VALU row and column passes in FP64 instead
//        of FP64 MFMA products (the same sums in another order).
template <int WS, bool BF16, int SHAPE, bool QREG = false, bool VDFT = false>
__device__ __forceinline__ void process_window_mixed(const KParams &p, const KJob &j, int bi, int bj,
                                                     long long win_local, char *wlds, const char *glds) {
    using LL = MixedLds<WS>;
    const double *Sl = (const double *)glds;
    const float *qdl = (const float *)(glds + LL::offQd);
    const float *twl = (const float *)(glds + LL::offTw);
    const double *tab = (const double *)(glds + LL::offTab);
    constexpr int W = 2 * WS;
    constexpr int QPL = WS * WS / 64;
    constexpr int NPOS = WS * WS;
    // derived per window: keeps lane-derived addressing from being hoisted out
    // of the persistent loop and kept live (in VGPRs) across all windows
    const int lane = fresh_lane();
    // lane L owns the positions k = L / WS + KSTEP t (t < QPL), l = L % WS
    constexpr int KSTEP = 64 / WS;
    const int lam = lane % WS;
    const int krow = lane / WS;
    const double *dft = tab;           // [WS][2] exp(-2 pi i k / WS)
    const double *ew = tab + 2 * WS;   // [W][2]  exp(+2 pi i k / W)

    // wave-uniform: the class's table bases stay in scalar registers
    const int cls = __builtin_amdgcn_readfirstlane(j.rowcls[bi] * j.ncolk + j.colcls[bj]);
    const unsigned char *tb = j.tables + (size_t)cls * p.lay.stride;
    const double *qD64 = (const double *)(tb + p.lay.offQD64);
    const double *invD = (const double *)(tb + p.lay.offInvD);
    const signed char *codes = (const signed char *)(tb + p.lay.offCodes);

    double *X = (double *)wlds;
    signed char *Cd = (signed char *)(wlds + LL::offCodes);
    C2<double> *stage = (C2<double> *)(wlds + LL::offStage);  // VALU and split-BF16 DFTs only

    wave_lds_fence();

    // ---- gather the sensor tile, weighted (absent pixels -> 0) -------------
    const int rs = (p.B * bi - p.off) / 2;
    const int cs = (p.B * bj - p.off) / 2;
    double e0 = 0.0;
    for (int m = fresh_lane(); m < NPOS; m += 64) {
        const int ip = m / WS, jp = m % WS;
        const int gi = rs + ip, gj = cs + jp;
        signed char code = codes[m];
        double x = 0.0;
        if (code >= 0 && gi >= 0 && gi < j.Ms && gj >= 0 && gj < j.Ns) {
            const double yv = load_measurement(j, (size_t)gi * j.Ns + gj);
            x = p.c.w[m] * yv;
            e0 += x * yv;
        } else {
            code = -1;
        }
        X[m] = x;
        Cd[m] = code;
    }
    e0 = uniform_f64(wave_sum(e0));
    wave_lds_fence();

    // ---- FP64 orientation-masked DFT of the window --------------------------
    C2<double> P[QPL][4];
    if constexpr (WS == 16 && !VDFT) {
        double Pre[4][4], Pim[4][4];
        if constexpr (BF16) dft16_splitbf16<double>(X, Cd, dft, (float *)stage, Pre, Pim);
        else dft16_mfma<double>(X, Cd, dft, Pre, Pim);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int o = 0; o < 4; ++o) P[t][o] = {Pre[t][o], Pim[t][o]};
    } else {
#pragma unroll
        for (int o = 0; o < 4; ++o) {  // unrolled: P must be indexed statically
#pragma unroll 1
            for (int s = 0; s < QPL; ++s) {
                const int ip = krow + KSTEP * s;
                C2<double> acc = {0.0, 0.0};
#pragma unroll 4
                for (int jp = 0; jp < WS; ++jp) {
                    const double x = (Cd[ip * WS + jp] == o) ? X[ip * WS + jp] : 0.0;
                    const int k = (jp * lam) & (WS - 1);
                    acc.re += x * dft[2 * k];
                    acc.im += x * dft[2 * k + 1];
                }
                stage[ip * WS + lam] = acc;
            }
            wave_lds_fence();
#pragma unroll
            for (int t = 0; t < QPL; ++t) {
                const int kap = krow + KSTEP * t;
                C2<double> acc = {0.0, 0.0};
#pragma unroll 4
                for (int ip = 0; ip < WS; ++ip) {
                    const C2<double> a = stage[ip * WS + lam];
                    const int k = (ip * kap) & (WS - 1);
                    const double tr = dft[2 * k], ti = dft[2 * k + 1];
                    acc.re += a.re * tr - a.im * ti;
                    acc.im += a.re * ti + a.im * tr;
                }
                P[t][o] = acc;
            }
            wave_lds_fence();
        }
    }

    const int lam_l = fresh_lane() % WS;
    const C2<float> tl = {(float)ew[2 * lam_l], (float)-ew[2 * lam_l + 1]};
    // the L-pixel response table, read with wave-uniform indices: scalar loads
    const CDouble *Ht = (const CDouble *)p.c.H;
    const CDouble *invDs = (const CDouble *)invD;

    const int BB = p.B * p.B;  // 16 or 64: divides the wavefront
    const int lgB = p.B == 8 ? 3 : 2;  // the block side is 4 or 8
    double outacc = 0.0;
    double E = e0;
    int nu_done = 0;
    // Eq. (18) over the picks kept so far (their coefficient step and
    // frequency, in this wavefront's w*y and code arrays, free after the
    // prologue): lane L sums output pixel L % BB over picks L / BB,
    // L / BB + 64 / BB, ...; the parts of a pixel are then added across the
    // lanes BB apart.
    C2<double> *pk = (C2<double> *)X;
    int16_t *pidx = (int16_t *)Cd;
    constexpr int PCAP = NPOS / 2;
    int npk = 0;
    auto add_picks = [&]() {
        wave_lds_fence();
        // the output pixel's coordinates, recomputed here (this runs once or a
        // few times per window) rather than held in registers through the loop
        const int ln = fresh_lane();
        const int xo = p.off + ((ln & (BB - 1)) >> lgB), yo = p.off + (ln & (p.B - 1));
        double acc = 0.0;
        for (int k = ln >> (2 * lgB); k < npk; k += 64 / BB) {
            const int f = pidx[k];
            const C2<double> g = pk[k];
            const int ph = (xo * (f / W) + yo * (f % W)) & (W - 1);
            acc += g.re * ew[2 * ph] - g.im * ew[2 * ph + 1];
        }
        for (int s = BB; s < 64; s <<= 1) acc += __shfl_xor(acc, s);
        outacc += acc;
        npk = 0;
        wave_lds_fence();
    };
    float4 q4r[QREG ? QPL : 1], t4r[QREG ? QPL : 1];
    if constexpr (QREG) {
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
            q4r[t] = *(const float4 *)(qdl + (t * 64 + lane) * 4);
            t4r[t] = *(const float4 *)(twl + (t * 64 + lane) * 4);
        }
    }

#pragma unroll 1
    for (int nu = 0; nu < p.iters; ++nu) {
        // Issue priority among the wavefronts of a SIMD rises with the
        // progress through an iteration: the projection at 0, the dependent
        // chain from the wave maximum to the step (reductions, readlanes, the
        // table reads that wait for the pick, little to overlap) at 2, the
        // rest of the iteration and the update at 1. Wavefronts in the bulk
        // work fill the gaps of the one in its chain.
        __builtin_amdgcn_s_setprio(0);
        // eq. (11) in FP32 for the lane's frequencies; per-lane largest and
        // second-largest key (metric bits, in-lane code in the low 4 bits)
        unsigned kb = 0u, ks = 0u;
        // per-lane q/D and twiddles of a position are read from LDS as the
        // position is projected (no read-ahead: its registers are worth more
        // as room for a fourth wavefront per SIMD, which hides the latency)
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
            float4 q4, t4;
            if constexpr (QREG) {
                q4 = q4r[t];
                t4 = t4r[t];
            } else {
                q4 = *(const float4 *)(qdl + (t * 64 + lane) * 4);
                t4 = *(const float4 *)(twl + (t * 64 + lane) * 4);
            }
            C2<float> Pf[4], R[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) Pf[o] = {(float)P[t][o].re, (float)P[t][o].im};
            project4_f32<SHAPE>(Pf, tl, C2<float>{t4.x, t4.y}, C2<float>{t4.z, t4.w}, R);
            const float qd[4] = {q4.x, q4.y, q4.z, q4.w};
            unsigned key[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float m = fmaf(R[c].re, R[c].re, R[c].im * R[c].im) * qd[c];
                key[c] = (__float_as_uint(m) & ~15u) | (unsigned)(t * 4 + c);
            }
            // top two of {kb, ks, a, b}: the second is max(ks, med3(kb, a, b))
            ks = max(ks, umed3(kb, key[0], key[1]));
            kb = umax3(kb, key[0], key[1]);
            ks = max(ks, umed3(kb, key[2], key[3]));
            kb = umax3(kb, key[2], key[3]);
            __builtin_amdgcn_sched_barrier(0);  // one position at a time: bounds register pressure
        }
        __builtin_amdgcn_s_setprio(2);
        // The FP32 winner stands when no other key reaches (1 - NEAR_TIE) of
        // it: exactly one lane's best and no lane's second are at or above it.
        const unsigned M = wave_max_u32(kb);
        const unsigned thr = __float_as_uint(__uint_as_float(M & ~15u) * (1.0f - NEAR_TIE));
        const unsigned long long hi1 = __ballot(kb >= thr);
        const unsigned long long hi2 = __ballot(ks >= thr);
        int idx;
        if (__popcll(hi1) == 1 && hi2 == 0ull) {
            const int L = __builtin_ctzll(hi1);
            const int code = (int)(M & 15u);
            const int t = code >> 2, a = (code >> 1) & 1, b = code & 1;
            idx = ((L / WS) + KSTEP * t + WS * a) * W + (L % WS) + WS * b;
        } else {
            // near tie: decide in FP64 from the FP64 state. The lane index is
            // derived afresh here, so that none of this (rare) branch's
            // addressing is computed ahead of the loop and kept in registers.
            const int ln = fresh_lane();
            const int krow_t = ln / WS, lam_t = ln % WS;
            double b0 = -1.0, b1 = -1.0;
            int i0 = 0, i1 = 0;
#pragma unroll
            for (int t = 0; t < QPL; ++t) {
                const int kap = krow_t + KSTEP * t;
                const C2<double> dtk = {ew[2 * kap], -ew[2 * kap + 1]};
                const C2<double> dtkl = {ew[2 * (kap + lam_t)], -ew[2 * (kap + lam_t) + 1]};
                const C2<double> dtl = {ew[2 * lam_t], -ew[2 * lam_t + 1]};
                C2<double> R[4];
                project4<double, SHAPE>(P[t], dtl, dtk, dtkl, R);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int a = c >> 1, b = c & 1;
                    const int f = (kap + WS * a) * W + lam_t + WS * b;
                    const double m = (R[c].re * R[c].re + R[c].im * R[c].im) * qD64[f];
                    if (a == 0) tie_keep<double>(b0, i0, m, f, TIE_REL);
                    else tie_keep<double>(b1, i1, m, f, TIE_REL);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            double best = b0;
            idx = i0;
            tie_merge<double>(best, idx, b1, i1, TIE_REL);
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o);
                const int oid = __shfl_xor(idx, o);
                tie_merge<double>(best, idx, ob, oid, TIE_REL);
            }
        }
        idx = __builtin_amdgcn_readfirstlane(idx);
        const int u = idx / W, v = idx % W;

        // L-pixel responses H_o(u, v) of the selected basis function (FP64)
        double Hr[4], Hi[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            Hr[o] = Ht[(size_t)idx * 8 + 2 * o];
            Hi[o] = Ht[(size_t)idx * 8 + 2 * o + 1];
        }

        // R_uv = sum_o conj(H_o(u, v)) P_o in FP64, from the owner lane
        const int ku = u & (WS - 1), lv = v & (WS - 1);
        const int tu = ku / KSTEP;
        const int owner = (ku % KSTEP) * WS + lv;
        double rr = 0.0, ri = 0.0;
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
            if (tu == t) {
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    rr = fma(Hr[o], P[t][o].re, fma(Hi[o], P[t][o].im, rr));
                    ri = fma(Hr[o], P[t][o].im, fma(-Hi[o], P[t][o].re, ri));
                }
            }
        }
        rr = readlane_f64(rr, owner);
        ri = readlane_f64(ri, owner);

        // eqs. (15)-(16), and the energy of eq. (8) where a floor is set, FP64
        const double id = invDs[idx];
        const double gr = p.gamma * id * rr, gi = p.gamma * id * ri;
        __builtin_amdgcn_s_setprio(1);
        bool stop = false;
        if (p.tau > 0.0) {
            E = uniform_f64(E - p.ecoef * (rr * rr + ri * ri) * id);
            // the floor is formed here, from an opaque copy of e0, so that it
            // is not computed ahead and carried through the loop in vector
            // registers (which would spill at four wavefronts per SIMD)
            double e0c = e0;
            asm volatile("" : "+v"(e0c));
            stop = E <= uniform_f64(p.tau * e0c);
        }
        // the spectra of the first orientation of the update, at the lane's
        // shifted positions, are read from LDS now, so that their latency
        // overlaps the pick record and the stopping test
        // lane coordinates recomputed here (a fresh lane index, then two
        // instructions) rather than held in registers through the loop
        const int lnu = fresh_lane();
        const int krow_u = lnu / WS, lam_u = lnu % WS;
        const C2<double> *Sc = (const C2<double> *)Sl + ((lam_u - lv) & (WS - 1));
        int srow[QPL];
#pragma unroll
        for (int t = 0; t < QPL; ++t) srow[t] = ((krow_u + KSTEP * t - ku) & (WS - 1)) * WS;
        C2<double> sn[QPL];
#pragma unroll
        for (int t = 0; t < QPL; ++t) sn[t] = Sc[srow[t]];
        __builtin_amdgcn_sched_barrier(0);
        // eq. (18): keep the pick; the central block is summed over the kept
        // picks when the stage is full and after the last iteration
        if (lane == 0) {
            pk[npk] = {gr, gi};
            pidx[npk] = (int16_t)idx;
        }
        if (++npk == PCAP) add_picks();
        if (j.sel != nullptr && lane == 0) ((GInt16 *)j.sel)[win_local * p.iters + nu] = (int16_t)idx;
        nu_done = nu + 1;
        if (stop) break;
        if (nu + 1 == p.iters) break;

        // eq. (17), factorised: P_o(k, l) -= g_o S_o(k - u, l - v) with
        // g_o = gamma delta H_o(u, v) (wave-uniform), orientation by
        // orientation (one coefficient live at a time); the spectra of
        // orientation o + 1 are read while orientation o is updated
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            C2<double> so[QPL];
#pragma unroll
            for (int t = 0; t < QPL; ++t) so[t] = o == 0 ? sn[t] : Sc[o * NPOS + srow[t]];
            const double gre = fma(gr, Hr[o], -gi * Hi[o]), gim = fma(gr, Hi[o], gi * Hr[o]);
#pragma unroll
            for (int t = 0; t < QPL; ++t) {
                P[t][o].re = fma(-gre, so[t].re, fma(gim, so[t].im, P[t][o].re));
                P[t][o].im = fma(-gre, so[t].im, fma(-gim, so[t].re, P[t][o].im));
            }
        }
    }
    if (npk > 0) add_picks();
    const int lo = fresh_lane();
    if (j.sel != nullptr)
        for (int nu = nu_done + lo; nu < p.iters; nu += 64) j.sel[win_local * p.iters + nu] = -1;
    if (lo < BB) {
        float *O = (float *)j.out;
        const int oi = lo >> lgB, oj = lo & (p.B - 1);
        const size_t row = (size_t)(p.B * bi + oi);
        O[row * (size_t)(2 * j.Ns) + (size_t)(p.B * bj + oj)] = (float)outacc;
    }
}

// Stage a class's FP64 spectra and per-lane q/D into LDS (whole workgroup);
// with `with_tab` also the class-independent twiddles.
template <int WS>
__device__ __forceinline__ void stage_tables(const KParams &p, const KJob &j, int cls, char *glds, bool with_tab) {
    using LL = MixedLds<WS>;
    constexpr int NPOS = WS * WS, W = 2 * WS, QPL = NPOS / 64;
    double *Sl = (double *)glds;
    float *qdl = (float *)(glds + LL::offQd);
    const unsigned char *tb = j.tables + (size_t)cls * p.lay.stride;
    const double *S64 = (const double *)(tb + p.lay.offS);
    const float *qD32 = (const float *)(tb + p.lay.offQD32);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));  // not hoisted out of the persistent loop
    // table order [pos][o][re, im] -> LDS order [o][pos][re, im]: for a fixed o the
    // lanes of a row read consecutive 16-byte entries (no bank conflicts)
    for (int e = tid; e < NPOS * 8; e += blockDim.x) {
        const int pos = e >> 3, o = (e >> 1) & 3, c = e & 1;
        Sl[(o * NPOS + pos) * 2 + c] = S64[e];
    }
    // q/D of the 4 frequencies (k + Ws a, l + Ws b) of each lane's positions
    for (int e = tid; e < QPL * 64 * 4; e += blockDim.x) {
        const int c = e & 3, ln = (e >> 2) & 63, t = e >> 8;
        const int kap = (ln / WS) + (64 / WS) * t, lam = ln % WS;
        qdl[e] = qD32[(kap + WS * (c >> 1)) * W + lam + WS * (c & 1)];
    }
    if (with_tab) {
        float *twl = (float *)(glds + LL::offTw);
        double *tab = (double *)(glds + LL::offTab);
        for (int e = tid; e < 2 * WS; e += blockDim.x) tab[e] = p.c.dft[e];
        for (int e = tid; e < 4 * WS; e += blockDim.x) tab[2 * WS + e] = p.c.ew[e];
        // e^{-i theta k} and e^{-i theta (k + l)} per lane position
        for (int e = tid; e < QPL * 64; e += blockDim.x) {
            const int ln = e & 63, t = e >> 6;
            const int kap = (ln / WS) + (64 / WS) * t, lam = ln % WS;
            twl[e * 4 + 0] = (float)p.c.ew[2 * kap];
            twl[e * 4 + 1] = (float)-p.c.ew[2 * kap + 1];
            twl[e * 4 + 2] = (float)p.c.ew[2 * (kap + lam)];
            twl[e * 4 + 3] = (float)-p.c.ew[2 * (kap + lam) + 1];
        }
    }
}

// One window per workgroup (used for selection diagnostics).
template <int WS, bool BF16, int SHAPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void mixed_window_kernel(KParams p, KJob j) {
    extern __shared__ __align__(16) char lds[];
    using L = MixedLds<WS>;
    const long long w = blockIdx.x;
    const long long nwin = (long long)j.nbi * j.nbj;
    if (w >= nwin) return;
    const int bi = (int)(w / j.nbj), bj = (int)(w % j.nbj);
    stage_tables<WS>(p, j, j.rowcls[bi] * j.ncolk + j.colcls[bj], lds, true);
    __syncthreads();
    process_window_mixed<WS, BF16, SHAPE>(p, j, bi, bj, w, lds + L::shared_bytes, lds);
}

// Persistent: workgroups pull groups of up to NW same-class windows. The
// group list is ordered by spatial tile and cut into XCD_RANGES contiguous
// ranges with one counter each; a workgroup drains the range of its own XCD
// (workgroups are dealt to the XCDs round-robin) and then the others, so the
// measurements and output lines of a tile stay in one XCD's L2. A claim takes
// `chunk` consecutive groups of a range (runs of one class inside a tile), and
// the class tables are staged into LDS only when the class changes. Every
// group index is claimed exactly once whatever the actual placement.
template <int WS, int NW, bool BF16, int SHAPE, bool QREG, bool VDFT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(QREG ? 2 : (VDFT || BF16) ? 3 : 4))) void
mixed_persistent_kernel(
    KParams p, const KJob *__restrict__ jobs, const WinGroup *__restrict__ groups, const int *__restrict__ range_begin,
    unsigned int *counters, int chunk) {
    extern __shared__ __align__(16) char lds[];
    using L = MixedLds<WS>;
    int *slot = (int *)(lds + L::offSlot);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    char *wl = lds + L::shared_bytes + (size_t)wave * L::wave_bytes(VDFT || BF16);
    const int home = (int)(blockIdx.x % XCD_RANGES);
    int tried = 0;             // ranges found exhausted (thread 0 only)
    int next = 0, left = 0;    // the current claim (thread 0 only)
    int staged_job = -1, staged_cls = -1;
    bool first = true;
    for (;;) {
        if (threadIdx.x == 0) {
            int g = -1;
            while (left == 0 && tried < XCD_RANGES) {
                const int r = (home + tried) % XCD_RANGES;
                const int n = range_begin[r + 1] - range_begin[r];
                const int k = (int)atomicAdd(counters + r, (unsigned)chunk);
                if (k < n) {
                    next = range_begin[r] + k;
                    left = min(chunk, n - k);
                } else {
                    ++tried;
                }
            }
            if (left > 0) {
                g = next++;
                --left;
            }
            *slot = g;
        }
        __syncthreads();
        // the group index is workgroup-uniform: keep it (and all that derives
        // from it) in scalar registers
        const int gi = __builtin_amdgcn_readfirstlane(*slot);
        if (gi < 0) break;
        const int gjob = groups[gi].job, gcount = groups[gi].count;
        const KJob J = jobs[gjob];
        const int w0 = groups[gi].win[0];
        const int cls = __builtin_amdgcn_readfirstlane(J.rowcls[w0 / J.nbj] * J.ncolk + J.colcls[w0 % J.nbj]);
        if (gjob != staged_job || cls != staged_cls) {
            stage_tables<WS>(p, J, cls, lds, first);
            first = false;
            staged_job = gjob;
            staged_cls = cls;
        }
        __syncthreads();
        if (wave < gcount) {
            const int lw = __builtin_amdgcn_readfirstlane(groups[gi].win[wave]);
            process_window_mixed<WS, BF16, SHAPE, QREG, VDFT>(p, J, lw / J.nbj, lw % J.nbj, lw, wl, lds);
        }
        __syncthreads();
    }
}

static size_t mixed_lds_bytes(int ws, int nw, bool bf16) {
    return ws == 16 ? MixedLds<16>::bytes(nw, bf16) : MixedLds<8>::bytes(nw, bf16);
}

template <int SHAPE>
static int launch_mw(const KParams &p, const KJob &job, int ws, void *stream) {
    const long long nwin = (long long)job.nbi * job.nbj;
    if (nwin <= 0) return 0;
    const size_t lds = mixed_lds_bytes(ws, 1, p.dft_bf16 != 0);
    const dim3 grid((unsigned)nwin), block(64);
    if (ws == 16 && p.dft_bf16 && SHAPE == SHAPE_THREE_QUARTER)
        mixed_window_kernel<16, true, SHAPE_THREE_QUARTER><<<grid, block, lds, (hipStream_t)stream>>>(p, job);
    else if (ws == 16)
        mixed_window_kernel<16, false, SHAPE><<<grid, block, lds, (hipStream_t)stream>>>(p, job);
    else
        mixed_window_kernel<8, false, SHAPE><<<grid, block, lds, (hipStream_t)stream>>>(p, job);
    return (int)hipGetLastError();
}

// Shapes with kernels: three-quarter and quarter sampling (the host rejects
// others, and the split-BF16 DFT with quarter sampling, before launching).
int launch_mixed_window(const KParams &p, const KJob &job, int ws, void *stream) {
    return p.shape == SHAPE_QUARTER ? launch_mw<SHAPE_QUARTER>(p, job, ws, stream)
                                    : launch_mw<SHAPE_THREE_QUARTER>(p, job, ws, stream);
}

template <int WS, int NW, bool BF16, int SHAPE, bool QREG, bool VDFT>
static int launch_mp(const KParams &p, const KJob *d_jobs, const WinGroup *d_groups, const int *range_begin,
                     unsigned int *counters, int chunk, int grid, void *stream) {
    const size_t lds = MixedLds<WS>::bytes(NW, VDFT || BF16);
    mixed_persistent_kernel<WS, NW, BF16, SHAPE, QREG, VDFT><<<dim3(grid), dim3(64 * NW), lds, (hipStream_t)stream>>>(
        p, d_jobs, d_groups, range_begin, counters, chunk);
    return (int)hipGetLastError();
}

template <int WS, bool BF16, int SHAPE, bool QREG, bool VDFT>
static int launch_mp_nw(const KParams &p, const KJob *d_jobs, const WinGroup *d_groups, const int *range_begin,
                        unsigned int *counters, const MixedVariant &v, int grid, void *stream) {
    if (v.nw == 1)
        return launch_mp<WS, 1, BF16, SHAPE, QREG, VDFT>(p, d_jobs, d_groups, range_begin, counters, v.chunk, grid,
                                                         stream);
    if (v.nw == 2)
        return launch_mp<WS, 2, BF16, SHAPE, QREG, VDFT>(p, d_jobs, d_groups, range_begin, counters, v.chunk, grid,
                                                         stream);
    return launch_mp<WS, 4, BF16, SHAPE, QREG, VDFT>(p, d_jobs, d_groups, range_begin, counters, v.chunk, grid,
                                                     stream);
}

// The knobs exist for W = 32 without the split-BF16 DFT; other plans run the
// default variant.
template <int SHAPE>
static int launch_mp_knobs(const KParams &p, const KJob *d_jobs, const WinGroup *d_groups, const int *range_begin,
                           unsigned int *counters, const MixedVariant &v, int grid, void *stream) {
    if (v.qreg && v.vdft)
        return launch_mp_nw<16, false, SHAPE, true, true>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
    if (v.qreg)
        return launch_mp_nw<16, false, SHAPE, true, false>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
    if (v.vdft)
        return launch_mp_nw<16, false, SHAPE, false, true>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
    return launch_mp_nw<16, false, SHAPE, false, false>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
}

int launch_mixed_persistent(const KParams &p, const KJob *d_jobs, const WinGroup *d_groups, const int *range_begin,
                            unsigned int *counters, int ws, const MixedVariant &v, int grid, void *stream) {
    constexpr int TQ = SHAPE_THREE_QUARTER, QS = SHAPE_QUARTER;
    if (v.nw != 1 && v.nw != 2 && v.nw != 4) return (int)hipErrorInvalidValue;
    if (v.chunk < 1) return (int)hipErrorInvalidValue;
    if (ws == 16 && p.dft_bf16)
        return launch_mp_nw<16, true, TQ, false, false>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
    if (ws == 16)
        return p.shape == QS ? launch_mp_knobs<QS>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream)
                             : launch_mp_knobs<TQ>(p, d_jobs, d_groups, range_begin, counters, v, grid, stream);
    return p.shape == QS ? launch_mp_nw<8, false, QS, false, false>(p, d_jobs, d_groups, range_begin, counters, v,
                                                                     grid, stream)
                         : launch_mp_nw<8, false, TQ, false, false>(p, d_jobs, d_groups, range_begin, counters, v,
                                                                     grid, stream);
}

template <int WS, int NW, bool QREG, bool VDFT>
static int occ_mp(int *blocks) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, mixed_persistent_kernel<WS, NW, false, SHAPE_THREE_QUARTER, QREG, VDFT>, 64 * NW,
        MixedLds<WS>::bytes(NW, VDFT));
}

template <bool QREG, bool VDFT>
static int occ_knobs(int ws, int nw, int *blocks) {
    if (ws == 16)
        return nw == 1 ? occ_mp<16, 1, QREG, VDFT>(blocks) : nw == 2 ? occ_mp<16, 2, QREG, VDFT>(blocks)
                                                                     : occ_mp<16, 4, QREG, VDFT>(blocks);
    return nw == 1 ? occ_mp<8, 1, false, false>(blocks) : nw == 2 ? occ_mp<8, 2, false, false>(blocks)
                                                                  : occ_mp<8, 4, false, false>(blocks);
}

// Occupancy of the three-quarter instantiation (the quarter-sampling one uses
// no more registers or LDS).
int mixed_blocks_per_cu(int ws, const MixedVariant &v, int *blocks) {
    if (v.qreg && v.vdft) return occ_knobs<true, true>(ws, v.nw, blocks);
    if (v.qreg) return occ_knobs<true, false>(ws, v.nw, blocks);
    if (v.vdft) return occ_knobs<false, true>(ws, v.nw, blocks);
    return occ_knobs<false, false>(ws, v.nw, blocks);
}

// ---------------------------------------------------------------------------
// Allocation-free single-image launch
// ---------------------------------------------------------------------------

// Work memory of the allocation-free launch: COUNTERS work counters at 0, the
// group ranges at NOALLOC_OFF_RANGES, the job at NOALLOC_OFF_JOB and the work
// list at NOALLOC_OFF_GROUPS. Each GPU holds its own copy until the process
// ends; host code reaches it only through the address noalloc_scratch returns.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
static_assert(sizeof(KJob) <= NOALLOC_OFF_GROUPS - NOALLOC_OFF_JOB, "job slot too small");
static_assert((XCD_RANGES + 1) * sizeof(int) <= NOALLOC_OFF_JOB - NOALLOC_OFF_RANGES, "range slot too small");
static_assert(COUNTERS * sizeof(unsigned int) <= NOALLOC_OFF_RANGES, "counter slot too small");

struct NoallocRanges {
    int r[XCD_RANGES + 1];
};

// Writes the job, the group ranges and zeroed work counters (one wavefront).
__global__ void noalloc_setup_kernel(KJob job, NoallocRanges rg, unsigned char *scr) {
    const int t = threadIdx.x;
    if (t < COUNTERS) ((unsigned int *)scr)[t] = 0u;
    if (t <= XCD_RANGES) ((int *)(scr + NOALLOC_OFF_RANGES))[t] = rg.r[t];
    if (t == 0) *(KJob *)(scr + NOALLOC_OFF_JOB) = job;
}

constexpr int NOALLOC_MAX_DEVICES = 64;
static unsigned char *g_scratch_addr[NOALLOC_MAX_DEVICES];

// The caller holds the library lock, so the table needs no lock of its own.
int noalloc_scratch(int dev, unsigned char **ptr) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    if (!g_scratch_addr[dev]) {
        void *a = nullptr;
        const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_scratch_addr[dev] = (unsigned char *)a;
    }
    *ptr = g_scratch_addr[dev];
    return 0;
}

int launch_mixed_noalloc(const KParams &p, const KJob &job, const WinGroup *host_groups, int ngroups,
                         const int *ranges, bool upload, int ws, const MixedVariant &v, int grid,
                         unsigned char *scr, void *stream) {
    if (ngroups < 0 || ngroups > NOALLOC_MAX_GROUPS) return (int)hipErrorInvalidValue;
    if (upload && ngroups > 0) {
        const hipError_t e = hipMemcpyAsync(scr + NOALLOC_OFF_GROUPS, host_groups, sizeof(WinGroup) * ngroups,
                                            hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e != hipSuccess) return (int)e;
    }
    NoallocRanges rg;
    for (int r = 0; r <= XCD_RANGES; ++r) rg.r[r] = ranges[r];
    noalloc_setup_kernel<<<dim3(1), dim3(64), 0, (hipStream_t)stream>>>(job, rg, scr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    return launch_mixed_persistent(p, (const KJob *)(scr + NOALLOC_OFF_JOB),
                                   (const WinGroup *)(scr + NOALLOC_OFF_GROUPS),
                                   (const int *)(scr + NOALLOC_OFF_RANGES), (unsigned int *)scr, ws, v, grid,
                                   stream);
}

}  // namespace ljsde
