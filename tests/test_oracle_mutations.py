"""Mutation check of the oracle's pins (CPU). Each entry plants one plausible
mistake in a temporary copy of the oracle: a flipped sign, a missing
conjugate, a transposition, a dropped factor, a shifted index, an ignored
mask. The pin suites (tests/test_oracle_pins.py, test_oracle_shapes.py,
test_oracle_weights.py) run against that copy and must fail, so that no such
mistake could pass them unnoticed. The real oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "ljsde_oracle.py")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_shapes.py", "tests/test_oracle_weights.py"]

# name: (text in the oracle, planted replacement)
MUTATIONS = {
    "phi_sign": ("e = np.exp(2j * np.pi * np.outer(n, n) / W)", "e = np.exp(-2j * np.pi * np.outer(n, n) / W)"),
    "phi_transposed": ("return e[:, None, :, None] * e[None, :, None, :]",
                       "return e[:, None, None, :] * e[None, :, :, None]"),
    "numerator_without_conjugate": ("R = a.conj().T @ (w * r)", "R = a.T @ (w * r)"),
    "quadrant_transposed": ("A[m, 2 * ip + a, 2 * jp + b] = 1.0", "A[m, 2 * ip + b, 2 * jp + a] = 1.0"),
    "block_offset": ("return (W - B) // 2\n", "return (W - B) // 2 - 2\n"),
    "window_origin": ("r0, c0 = B * bi - off, B * bj - off\n", "r0, c0 = B * bi - off + 2, B * bj - off\n"),
    "weight_centre": ("c = (W - 1) / 2.0", "c = W / 2.0"),
    "normaliser_without_weights": ("D = (w[:, None] * np.abs(a) ** 2).sum(axis=0)", "D = (np.abs(a) ** 2).sum(axis=0)"),
    "residual_update_sign": ("r = r - gamma * delta * a[:, k]", "r = r + gamma * delta * a[:, k]"),
    "C_transposed": ("C = Bm.T @ a", "C = (Bm.T @ a).T"),
    "projected_update_conjugated": ("R = R - gamma * delta * C[:, k]", "R = R - gamma * np.conj(delta) * C[:, k]"),
    "coefficient_without_gamma": ("tr.coeffs[k] += gamma * delta                        # eq. (15)\n        r =",
                                  "tr.coeffs[k] += delta\n        r ="),
    "validity_ignored": ("            if not valid[ip, jp]:\n                continue\n            o = int(codes[ip, jp])",
                         "            o = int(codes[ip, jp])"),
    "frequency_weight_not_symmetric": ("st = np.minimum(s, W - s).astype(np.float64)", "st = s.astype(np.float64)"),
    "synthesis_conjugated": ("f = Phi.reshape(W * W, W * W) @ coeffs", "f = Phi.reshape(W * W, W * W) @ np.conj(coeffs)"),
    "unobserved_step_divides": ("return R[k] / D[k] if obs[k] else 0.0", "return R[k] / D[k]"),
}


def _run_pins(tmp_path, oracle_src):
    """The pin suites against a copy of the oracle with the given source."""
    (tmp_path / "oracle").mkdir()
    (tmp_path / "oracle" / "__init__.py").write_text("")
    (tmp_path / "oracle" / "ljsde_oracle.py").write_text(oracle_src)
    shutil.copytree(os.path.join(ROOT, "synth"), tmp_path / "synth")
    (tmp_path / "tests").mkdir()
    for f in ["__init__.py", "conftest.py"] + [os.path.basename(p) for p in PINS]:
        shutil.copy(os.path.join(ROOT, "tests", f), tmp_path / "tests" / f)
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), tmp_path / "tests" / "golden")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                          cwd=tmp_path, capture_output=True, text=True, timeout=900)


def test_unmodified_copy_passes_the_pins(tmp_path):
    """Control: the copied layout itself passes, so a failure below is the
    planted mistake's."""
    r = _run_pins(tmp_path, open(ORACLE).read())
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    src = open(ORACLE).read()
    old, new = MUTATIONS[name]
    assert src.count(old) >= 1, f"mutation {name} no longer applies to the oracle"
    r = _run_pins(tmp_path, src.replace(old, new))
    assert r.returncode == 1, f"no pin fails with the planted mistake {name}: {r.stdout[-1000:]}"
    assert " failed" in r.stdout.strip().splitlines()[-1]   # a pin's assertion, not a collection error
