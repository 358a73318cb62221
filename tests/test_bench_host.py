"""Host logic of bench.py (no GPU): the one-GPU contract, the plain-method
flop count of the roofline, the roofline record, and the source hashes that
keep stored HBM traffic tied to the kernels it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

# rocksalt workload: n_max 6/4, basis 8/8, l_max 4, 50 hidden, D = 7 + 4 * 5
HP = {"n_species": 2, "n_max_radial": 6, "n_max_angular": 4, "basis_radial": 8, "basis_angular": 8,
      "hidden": 50, "dim": 27, "four_body": 0}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_reference_flop_count_by_hand():
    # per radial neighbour 2*7*9 + 4*9 + 20 = 182, per angular neighbour
    # 2*5*9 + 4*9 + 3*24 + 2*5*24 = 438, network 4*27*50 = 5400
    ref = bench.flops_per_atom_reference(HP, 90.0, 26.0)
    assert ref["descriptor"] == pytest.approx(90 * 182 + 26 * 438 + 5400)
    # radial force 2*(2*7*9 + 6*9) + 4*7 + 30 = 418; angular force 2*(4*5*9 + 10*24 + 8*5*24) = 2760
    assert ref["force"] == pytest.approx(90 * 418)
    assert ref["force_ang"] == pytest.approx(26 * 2760)


def test_roofline_record():
    units = 4096 * 32
    r = bench.roofline("descriptor", 90.0, HP, 90.0, 26.0, units, {})
    flop = bench.flops_per_atom_reference(HP, 90.0, 26.0)["descriptor"]
    ach = flop * units / 90e-6 / 1e12
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(ach, abs=1e-3)
    assert r["frac"] == pytest.approx(ach / 157.3, abs=1e-4)
    assert r["frac_of_non_packed_fp32"] == pytest.approx(2 * ach / 157.3, abs=1e-4)
    assert r["traffic"] is None
    # a kernel without a flop count is held against the HBM roofline by its algorithmic bytes
    h = bench.roofline("trpmd", 10.0, HP, 90.0, 26.0, units, {"trpmd": 108.0})
    assert h["bound"] == "hbm" and h["unit"] == "GB/s"
    assert h["achieved"] == pytest.approx(108.0 * units / 10e-6 / 1e9, abs=0.1)
    assert bench.roofline(None, 10.0, HP, 90.0, 26.0, units, {}) is None


def test_source_hashes():
    h = {k: bench.kernel_source_hash(k) for k in bench.KERNEL_SOURCES}
    assert all(len(v) == 16 and int(v, 16) >= 0 for v in h.values())
    # kernels of one file share a hash, kernels of different files do not
    assert h["descriptor"] == h["force"] == h["force_ang"] == h["reduce"]
    assert h["nlist"] == h["centroid"] != h["descriptor"]
    assert h["trpmd"] not in (h["descriptor"], h["nlist"])
    assert bench.kernel_source_hash("descriptor") == h["descriptor"]
