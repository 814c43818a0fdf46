"""Host-side checks of the benchmark script (no GPU): the one-GPU contract and
the code hash that keys the committed HBM-traffic records."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_code_hash_ignores_comments_and_blank_space():
    a = "int f(int x) {\n  return x + 1;  // step\n}\n"
    b = "/* header */\nint f(int x)\n{ return x + 1; }\n\n"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_traffic_record_is_used_only_for_the_code_it_was_taken_on(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_hash(["k.hip"])
    (tmp_path / "profiles" / "kernel_traffic.json").write_text(
        '{"w": {"kernel_hash": "%s", "hbm_bytes_per_launch": 123.0}}' % h)
    assert bench.load_traffic("w", ["k.hip"]) == 123.0
    assert bench.load_traffic("other", ["k.hip"]) is None
    src.write_text("// a comment changes nothing\n__global__ void k() {}\n")
    assert bench.load_traffic("w", ["k.hip"]) == 123.0
    src.write_text("__global__ void k() { int x = 0; }\n")
    assert bench.load_traffic("w", ["k.hip"]) is None


def test_divergence_counts_conjugate_partners_and_reports_the_first_gap():
    W = bench.W
    conj = lambda k: ((-(k // W)) % W) * W + (-(k % W)) % W  # noqa: E731
    picks = {(0, 0): [0, 5, 7], (0, 1): [3, 9, 2], (0, 2): [4, 4, 4]}
    gaps = {(0, 0): [0.5, 0.1, 0.2], (0, 1): [0.3, 1e-7, 0.4], (0, 2): [0.2, 0.2, 2e-6]}
    sel = {(0, 0): [0, 5, 7],                 # equal
           (0, 1): [3, conj(9), conj(2)],     # conjugate partners from the second pick on
           (0, 2): [4, 4, 6]}                 # a different frequency at the third pick
    dv = bench.divergence(lambda k: sel[k], picks, gaps)
    assert dv["diverged"] == 2
    assert dv["diverged_modulo_conjugation"] == 1
    g = dv["oracle_top2_gap_at_first_divergence"]
    assert g["min"] == 1e-7 and g["max"] == 2e-6
    assert bench.divergence(lambda k: picks[k], picks, gaps)["oracle_top2_gap_at_first_divergence"] is None



def test_cpu_baseline_spreads_its_sample_over_the_images_and_keys_it_by_image():
    """The oracle sample of a batch covers every image, and each block comes
    back under (image, block row, block column) with the oracle's own result."""
    from oracle import ljsde_oracle as O
    from synth import make_case
    imgs = [make_case(16, 16, 2, seed=3), make_case(12, 20, 4, seed=4)]
    rec, res, picks, gaps = bench.cpu_baseline([(c["y"], c["tile"], 0xE, None) for c in imgs], 4, 6, label="t")
    assert {k for k, _, _ in res} == {0, 1}
    assert len(res) == 6 and set(res) == set(picks) == set(gaps)
    for (k, bi, bj), blk in res.items():
        ref, tr = O.reconstruct(imgs[k]["y"], imgs[k]["tile"], iters=4, form="RL", blocks=[(bi, bj)], traces=True)
        assert abs(blk - ref[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4]).max() == 0.0
        assert list(picks[(k, bi, bj)]) == tr[(bi, bj)].picks
    assert rec["kind"] == "oracle" and rec["cores"] >= 1 and rec["value"] > 0
