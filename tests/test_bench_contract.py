"""The bench's command-line contract and byte model (CPU only: nothing here touches a GPU)."""

import json
import os
import subprocess
import sys
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _fake_ham(dim_up, dim_dn, w_up, w_dn, eb=2):
    sp = lambda d, w: types.SimpleNamespace(dim=d, width=w, entry_bytes=eb)
    return types.SimpleNamespace(dim=dim_up * dim_dn, dim_up=dim_up, dim_dn=dim_dn, up=sp(dim_up, w_up),
                                 dn=sp(dim_dn, w_dn))


def test_algorithmic_bytes_per_launch():
    """k_up 2pD + up table, k_down 4pD + down table + both bases, k_update 3pD (4pD mixed)."""
    h = _fake_ham(12870, 12870, 32, 32)
    D = 12870 * 12870
    b64 = bench.kernel_bytes(h, 8)
    assert b64["k_up"] == 2 * 8 * D + 12870 * 32 * 2
    assert b64["k_down"] == 4 * 8 * D + 12870 * 32 * 2 + 8 * 2 * 12870
    assert b64["k_update"] == 3 * 8 * D
    b32 = bench.kernel_bytes(h, 4)
    assert b32["k_update"] == 4 * 4 * D
    wide = bench.kernel_bytes(_fake_ham(48620, 48620, 24, 24, eb=4), 8)
    assert wide["k_up"] == 2 * 8 * 48620 ** 2 + 48620 * 24 * 4


def test_traffic_record_only_for_its_workload_and_basis_order():
    assert bench.measured_traffic("f64", "k_down", "some_other_workload", "hops") is None
    rec = json.load(open(os.path.join(ROOT, "paper_1511_00863_amd", "measured_traffic.json")))
    other = "ascending" if rec.get("basis_order_down", "ascending") == "hops" else "hops"
    assert bench.measured_traffic("f64", "k_down", rec["workload"], other) is None


def test_progress_lines_go_to_stderr(capsys):
    bench.progress("a block")
    out, err = capsys.readouterr()
    assert out == "" and "a block" in err


def test_down_basis_order_follows_the_lds_row_rule():
    """Hop-count order where FP64 rows (complex: pairs) fit the down part's LDS staging, ascending beyond."""
    args = types.SimpleNamespace(basis_order="hops")
    assert bench.dn_order_for(args, 12870) == "hops"                      # 4x4 torus, 8 per species
    assert bench.dn_order_for(args, bench.LDS_ROW_STATES) == "hops"
    assert bench.dn_order_for(args, bench.LDS_ROW_STATES + 1) == "ascending"
    assert bench.dn_order_for(args, 48620) == "ascending"                 # 18-site chain, 9 per species
    assert bench.dn_order_for(args, 8568, cplx=True) == "hops"            # 18-site checkerboard, 5 per species
    assert bench.dn_order_for(args, 12000, cplx=True) == "ascending"
    assert bench.dn_order_for(types.SimpleNamespace(basis_order="ascending"), 12870) == "ascending"
