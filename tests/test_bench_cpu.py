"""Host logic of bench.py, on the CPU: the roofline arithmetic, the traffic
table's source check, the point-group orbit count, and the one-GPU guard."""
import hashlib
import itertools
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _orbits_by_group(D, nk):
    """Orbit count by applying every element of the hyperoctahedral group
    (axis permutations times sign flips, 2^D D! elements) and keeping one
    representative per orbit: independent of the closed form in bench.py."""
    seen, orbits = set(), 0
    for q in itertools.product(range(nk), repeat=D):
        if q in seen:
            continue
        orbits += 1
        for perm in itertools.permutations(range(D)):
            for signs in itertools.product((1, -1), repeat=D):
                seen.add(tuple((signs[a] * q[perm[a]]) % nk for a in range(D)))
    return orbits


@pytest.mark.parametrize("D,nk", [(1, 64), (2, 8), (2, 32), (3, 8), (3, 16), (4, 4)])
def test_orbit_count_matches_group_action(D, nk):
    assert bench.orbit_count(D, nk) == _orbits_by_group(D, nk)


def test_orbit_counts_of_the_irreducible_wedges():
    # C4v on 32^2 and O_h on 16^3: the irreducible wedges of the square and
    # cubic Brillouin zones
    assert bench.orbit_count(2, 32) == 153
    assert bench.orbit_count(3, 16) == 165


class _FakeLib:
    def __init__(self, variant):
        self.variant = variant

    def df_ladder_variant(self, n_nu, prec):
        return self.variant


def test_roofline_arithmetic():
    n_om, N, n_nu, ms = 31, 1024, 64, 3.0
    flops = 2 * n_om * N * 8.0 * n_nu ** 3
    r = bench.roofline_of(0, _FakeLib("gjb_o4"), n_om, N, n_nu, ms)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["peak"] == 78.6
    assert r["algorithmic_flops_per_launch"] == flops
    assert r["achieved"] == pytest.approx(flops / 3e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["kernel"] == "k_ladder_gjb_f64_o4<64, true>"
    assert bench.kernel_symbol("gjb@p1", 128) == "k_ladder_gjb_f64<128, true, true>"
    assert bench.kernel_symbol("gjb", 96) == "k_ladder_gjb_f64_xk<96, true, 2>"
    assert bench.kernel_symbol("mixed", 96) == "k_ladder_mixed<96, true>"
    r = bench.roofline_of(2, _FakeLib("fp32_o4"), n_om, N, n_nu, ms)
    assert r["peak"] == 157.3 and r["algorithmic_flops_per_launch"] == flops
    # refined solve: 16 n^3 in FP32 and 8 n^3 in FP64, each at its own peak
    r = bench.roofline_of(1, _FakeLib("mixed_o3"), n_om, N, n_nu, ms)
    assert r["algorithmic_flops_per_launch"] == 3 * flops
    assert r["peak"] == pytest.approx(3.0 / (2.0 / 157.3 + 1.0 / 78.6))
    assert r["peak"] == pytest.approx(117.9, abs=0.05)


def test_traffic_table_applies_only_to_matching_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1507_00895_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "a.hip").write_bytes(b"kernel a")
    (csrc / "b.hpp").write_bytes(b"header b")
    digest = hashlib.sha256(b"kernel a" + b"header b").hexdigest()[:16]
    table = {"source_files": ["a.hip", "b.hpp"], "source_sha256_16": digest,
             "kernels": {"k<64>@300": {"traffic_bytes": 3.0e9}}}
    (tmp_path / "profiles" / "ladder_traffic.json").write_text(json.dumps(table))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k<64>", 300, 3) == pytest.approx(1.0e9)
    assert bench.measured_traffic("k<64>", 600, 3) is None      # other launch shape
    assert bench.measured_traffic("other<64>", 300, 3) is None
    (csrc / "a.hip").write_bytes(b"kernel a, edited")
    assert bench.measured_traffic("k<64>", 300, 3) is None      # sources changed


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_cpu_baseline_on_a_small_problem():
    from paper_1507_00895_amd import inputs as I
    p = I.atomic_limit_problem(2, 8, 16, 3, 10.0, 2.0, 0.1)
    out = bench.cpu_baseline([p], budget_s=0.5)
    assert out["kind"] == "oracle" and out["unit"] == "solves/s"
    assert out["value"] > 0 and out["single_process"]["value"] > 0
    # the core count is the number of processes that ran the ladder
    assert out["cores"] == out["processes"] == min(out["affinity_cores"], 16, p.n_om)
    assert out["single_process"]["cores"] == 1 and out["blas_threads_per_process"] == 1
    assert out["affinity_cores"] >= 1 and out["cpu_count"] >= 1
    assert "all 3 bosonic slices" in out["sample"]
