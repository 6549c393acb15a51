"""Host logic of the profile summaries (paper_1204_0111_amd/profile_summary.py)
on small synthetic rocprofv3 CSV files: the last-step selection, the copy
calibration of FETCH_SIZE / WRITE_SIZE and the per-XCD scaling of
GRBM_GUI_ACTIVE in the matrix-core busy fraction."""

import csv
import json

from paper_1204_0111_amd import profile_summary as ps

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_pmc_scales_by_the_copy_and_keeps_the_last_step(tmp_path):
    # dispatch 1: the 512 MiB calibration copy; 2: an earlier step's k_fwd
    # (ignored); 3: the velocity check opening the last step; 4, 5: k_fwd
    def rows(counter, copy_kib, vals):
        return [(1, 1 << 20, "__amd_rocclr_copyBuffer", counter, copy_kib),
                (2, 256, "void hsw::k_fwd<float, 1, 64, 256>(x)", counter, 999999.0),
                (3, 256, "hsw::k_check_velocity(x)", counter, 1.0),
                (4, 256, "void hsw::k_fwd<float, 1, 64, 256>(x)", counter, vals[0]),
                (5, 256, "void hsw::k_fwd<float, 1, 16, 512>(x)", counter, vals[1])]
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(f, rows("FETCH_SIZE", 262144.0, (100.0, 300.0)))   # reads half of the copied bytes
    _write(w, rows("WRITE_SIZE", 524288.0, (10.0, 30.0)))     # reads them all
    out = tmp_path / "s.txt"
    ps.pmc(str(f), str(w), "k_fwd", "toy", str(out), "cmd f", "cmd w")
    res = json.loads(open(out).read().strip().splitlines()[-1][len("result:"):])
    assert res["dispatches"] == 2
    assert abs(res["fetch_scale"] - 2.0) < 1e-12 and abs(res["write_scale"] - 1.0) < 1e-12
    assert abs(res["hbm_bytes_per_launch"] - (200.0 * 1024 * 2 + 20.0 * 1024)) < 1e-6


def test_sq_divides_the_active_cycles_by_the_xcds(tmp_path):
    # one dispatch: MFMA busy on every SIMD for half of one XCD's active cycles
    g = 8 * 1000.0   # summed over the eight XCDs
    rows = [(1, 256, "hsw::k_check_velocity(x)", "GRBM_GUI_ACTIVE", 1.0),
            (2, 256, "void hsw::k_update<float>(x)", "GRBM_GUI_ACTIVE", g),
            (2, 256, "void hsw::k_update<float>(x)", "SQ_VALU_MFMA_BUSY_CYCLES", 500.0 * ps.SIMDS),
            (2, 256, "void hsw::k_update<float>(x)", "SQ_WAVE_CYCLES", 100.0),
            (2, 256, "void hsw::k_update<float>(x)", "SQ_WAIT_INST_ANY", 25.0)]
    c = tmp_path / "c.csv"
    _write(c, rows)
    out = tmp_path / "sq.txt"
    ps.sq(str(c), "toy", str(out), "cmd")
    line = [l for l in open(out) if l.startswith("k_update")][0].split()
    assert line[2] == "50.0%" and line[3] == "0.250"


def test_last_step_families_start_at_the_last_velocity_check(tmp_path):
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [("void hsw::k_bwd_mm<float, 1, 4>(x)", 10, 20),      # an earlier step
            ("hsw::k_check_velocity(x)", 30, 31),
            ("void hsw::k_bwd_mm<float, 1, 16>(x)", 40, 50),
            ("void hsw::k_bwd_mm<float, 4, 4>(x)", 60, 90),
            ("void hsw::k_fwd_mm<float, 4, 4>(x)", 100, 105)]
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))
    fam = ps.last_step_families(str(p))
    assert fam["hsw::k_bwd_mm"] == (2, 40) and fam["hsw::k_fwd_mm"] == (1, 5)
