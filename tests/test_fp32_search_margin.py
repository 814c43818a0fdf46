"""Measured margin of the FP32 search's near-tie guard (CPU).

The FP32 plans keep the loop state P_o(k, l) (the factorised projected
residual: one (W/2)-point DFT of the weighted residual per pixel code) in
FP64, but evaluate the projection through the pixel responses, the eq. (11)
metric and the argmax in FP32, and accept the FP32 winner only when no other
metric reaches a relative 1e-4 of it (otherwise the iteration is re-decided
in FP64). This test replays that arithmetic on the CPU: an FP64 recurrent loop
in the factorised form (its selection sequences are checked against the
oracle's), and at every iteration the FP32 evaluation of all W^2 metrics from
the FP64 state, in the kernel's order of operations (rounding of P to float32,
the per-quadrant sums from two pair sums, the twiddle products folded into
the 2 x 2 Walsh-Hadamard step as fused multiply-adds (s1 = Q_0 + t_kl Q_3,
d1 = 2 Q_0 - s1, u1 = t_l Q_1, s2 = u1 + t_k Q_2, d2 = 2 u1 - s2), |R|^2 q / D
with q / D rounded to float32, the four low bits of the key replaced by the
frequency code). A fused multiply-add is replayed as the exact product and sum in
float64, rounded once more to float32. It asserts that every accepted FP32 decision
equals the FP64 decision, and measures the largest FP32 metric error relative
to the maximum metric among the candidates within 1e-3 of it: the guard's
margin is 1e-4 divided by twice that error.
"""
import numpy as np
import pytest

from oracle import ljsde_oracle as O
from synth import QUARTER, THREE_QUARTER, make_case

W, B, WS = 32, 4, 16
THETA = 2 * np.pi / W
NEAR_TIE = np.float32(1e-4)


def _responses(shape):
    """H_o(sigma, rho): the sum of e^{i theta (a sigma + b rho)} over the
    quadrants q = 2a + b that a pixel of code o integrates."""
    s = np.arange(W)
    H = np.zeros((4, W, W), dtype=np.complex128)
    for o in range(4):
        for q in range(4):
            if (shape >> (q ^ o)) & 1:
                H[o] += np.exp(1j * THETA * ((q >> 1) * s[:, None] + (q & 1) * s[None, :]))
    return H


def _fp32_keys(P, qd32, shape):
    """FP32 metrics (as keys with the 4 low bits cleared) of all W^2
    frequencies from the FP64 state P [4][WS][WS], in the kernel's order."""
    f32 = np.float32
    f64 = np.float64

    def fma(x, y, z):
        return (np.asarray(x, f64) * np.asarray(y, f64) + np.asarray(z, f64)).astype(f32)

    Pr = P.real.astype(f32)
    Pi = P.imag.astype(f32)
    if shape == THREE_QUARTER:
        # Q_q is the sum of the three orientations other than q, from two pair sums
        ar, ai = Pr[0] + Pr[1], Pi[0] + Pi[1]
        br, bi = Pr[2] + Pr[3], Pi[2] + Pi[3]
        Qr = [Pr[1] + br, Pr[0] + br, ar + Pr[3], ar + Pr[2]]
        Qi = [Pi[1] + bi, Pi[0] + bi, ai + Pi[3], ai + Pi[2]]
    else:
        Qr = [Pr[q] for q in range(4)]
        Qi = [Pi[q] for q in range(4)]
    k = np.arange(WS)
    ck = np.cos(THETA * k).astype(f32)[:, None]
    sk = (-np.sin(THETA * k)).astype(f32)[:, None]
    cl = np.cos(THETA * k).astype(f32)[None, :]
    sl = (-np.sin(THETA * k)).astype(f32)[None, :]
    ckl = np.cos(THETA * (k[:, None] + k[None, :])).astype(f32)
    skl = (-np.sin(THETA * (k[:, None] + k[None, :]))).astype(f32)

    two = f32(2)
    s1 = (fma(ckl, Qr[3], fma(-skl, Qi[3], Qr[0])), fma(ckl, Qi[3], fma(skl, Qr[3], Qi[0])))
    d1 = (fma(two, Qr[0], -s1[0]), fma(two, Qi[0], -s1[1]))
    u1 = (fma(cl, Qr[1], -(sl * Qi[1])), fma(cl, Qi[1], sl * Qr[1]))
    s2 = (fma(ck, Qr[2], fma(-sk, Qi[2], u1[0])), fma(ck, Qi[2], fma(sk, Qr[2], u1[1])))
    d2 = (fma(two, u1[0], -s2[0]), fma(two, u1[1], -s2[1]))
    R = {(0, 0): (s1[0] + s2[0], s1[1] + s2[1]), (0, 1): (d1[0] - d2[0], d1[1] - d2[1]),
         (1, 0): (d1[0] + d2[0], d1[1] + d2[1]), (1, 1): (s1[0] - s2[0], s1[1] - s2[1])}
    keys = np.zeros((W, W), dtype=f32)
    for (a, b), (rr, ri) in R.items():
        qd = qd32[WS * a:WS * a + WS, WS * b:WS * b + WS]
        m = fma(rr, rr, ri * ri) * qd
        # the key keeps the metric's upper bits; the low 4 bits carry the code
        keys[WS * a:WS * a + WS, WS * b:WS * b + WS] = (m.view(np.uint32) & np.uint32(~15 & 0xFFFFFFFF)).view(f32)
    return keys.reshape(-1)


def _run_window(y, tile, bi, bj, shape, iters=100, rho=0.7, gamma=0.5):
    y_loc, codes, valid = O.local_window(y, tile, bi, bj, W, B)
    w = O.spatial_weights(W, rho) * valid.reshape(-1)
    q = O.frequency_weights(W, "fsr").reshape(W, W)
    H = _responses(shape)
    X = (w * y_loc).reshape(WS, WS)
    cd = np.where(valid, codes, -1)
    P = np.stack([np.fft.fft2(np.where(cd == o, X, 0.0)) for o in range(4)])
    S = np.stack([np.fft.fft2(np.where(cd == o, w.reshape(WS, WS), 0.0)) for o in range(4)])
    D = np.einsum("osr,o->sr", np.abs(H) ** 2, S[:, 0, 0].real)
    obs = (D > 0) & (D > O.D_REL * D.max())
    qd = np.where(obs, q / np.where(obs, D, 1.0), 0.0)
    qd32 = qd.astype(np.float32)
    idx = np.arange(W)
    picks, accepted, fallbacks, worst = [], 0, 0, 0.0
    for _ in range(iters):
        Pf = P[:, idx[:, None] % WS, idx[None, :] % WS]        # [4][W][W]
        R = np.einsum("osr,osr->sr", np.conj(H), Pf)
        m64 = (qd * np.abs(R) ** 2).reshape(-1)
        best = m64.max()
        k64 = int(np.flatnonzero(m64 >= best * (1 - O.TIE_REL))[0]) if best > 0 else 0
        keys = _fp32_keys(P, qd32, shape)
        M = keys.max()
        thr = np.float32(M * (np.float32(1) - NEAR_TIE))
        near = np.flatnonzero(keys >= thr)
        if best > 0:
            cand = np.flatnonzero(m64 >= (1 - 1e-3) * best)
            worst = max(worst, float(np.max(np.abs(keys[cand].astype(np.float64) - m64[cand])) / best))
        if near.size == 1:
            accepted += 1
            assert int(near[0]) == k64, "an accepted FP32 decision differs from the FP64 one"
        else:
            fallbacks += 1
        picks.append(k64)
        u, v = divmod(k64, W)
        delta = R[u, v] / D[u, v] if obs[u, v] else 0.0
        g = gamma * delta * H[:, u, v]
        for o in range(4):
            P[o] -= g[o] * np.roll(np.roll(S[o], u % WS, axis=0), v % WS, axis=1)
    return picks, accepted, fallbacks, worst


@pytest.mark.parametrize("shape", [THREE_QUARTER, QUARTER], ids=["three_quarter", "quarter"])
def test_fp32_guard_margin(shape):
    c = make_case(128, 128, 4, seed=3, shape=shape)
    y, tile = c["y"], c["tile"]
    rng = np.random.default_rng(7)
    nb = 128 // B
    blocks = [tuple(map(int, divmod(int(f), nb))) for f in rng.choice(nb * nb, size=24, replace=False)]
    blocks += [(0, 0), (0, nb - 1), (nb - 1, 5)]  # border windows (clipped classes)
    _, tr = O.reconstruct(y, tile, W=W, B=B, iters=100, form="RL", blocks=blocks, traces=True, shape=shape)
    acc = fb = 0
    worst = 0.0
    for bi, bj in blocks:
        picks, a, f, wr = _run_window(y, tile, bi, bj, shape)
        assert picks == tr[(bi, bj)].picks, (bi, bj)   # the FP64 replay is the oracle's sequence
        acc, fb, worst = acc + a, fb + f, max(worst, wr)
    margin = float(NEAR_TIE) / (2 * worst)
    print(f"shape {shape:#x}: {acc} accepted FP32 decisions, {fb} FP64 re-decisions "
          f"({fb / (acc + fb):.2%}), largest relative FP32 metric error near the top {worst:.2e}, "
          f"guard margin {margin:.0f}x")
    assert acc > 0.9 * (acc + fb)
    assert margin >= 10
