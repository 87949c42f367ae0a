"""The text summaries committed under profiles/ (CPU only): mean counter values per
dispatch, and MFMA utilization = busy cycles summed over the SIMDs / (GPU cycles x SIMDs),
with GRBM_GUI_ACTIVE summed over the 8 XCDs."""
import csv

from paper_2101_12597_amd import profile_summary as P


def _write(path, rows):
    keys = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def _line(out, name):
    return next(l for l in out.splitlines() if l.startswith(name)).split()


def test_pmc_mean_per_dispatch(tmp_path, capsys):
    p = tmp_path / "c.csv"
    _write(p, [(1, "kern_a", "FETCH_SIZE", 100.0, 0, 1), (2, "kern_a", "FETCH_SIZE", 300.0, 0, 1),
               (3, "kern_b", "FETCH_SIZE", 50.0, 0, 1)])
    P.pmc_csv(str(p))
    out = capsys.readouterr().out
    a, b = _line(out, "kern_a"), _line(out, "kern_b")
    assert a[-2:] == ["2", "200.0"] and b[-2:] == ["1", "50.0"]


def test_mfma_utilization(tmp_path, capsys):
    # two dispatches of 1000 ns and 3000 ns; GPU cycles per dispatch = GRBM / 8 XCDs, and
    # 1024 SIMDs: util = busy / (GRBM / 8 * 1024) summed over the dispatches
    gui1, gui2 = 8 * 2000.0, 8 * 6000.0
    busy1, busy2 = 0.25 * 2000 * 1024, 0.5 * 6000 * 1024
    _write(tmp_path / "m.csv", [
        (1, "zkern", "SQ_VALU_MFMA_BUSY_CYCLES", busy1, 0, 1000), (1, "zkern", "GRBM_GUI_ACTIVE", gui1, 0, 1000),
        (2, "zkern", "SQ_VALU_MFMA_BUSY_CYCLES", busy2, 5000, 8000), (2, "zkern", "GRBM_GUI_ACTIVE", gui2, 5000, 8000)])
    P.mfma_csv(str(tmp_path / "m.csv"))
    row = _line(capsys.readouterr().out, "zkern")
    expect = 100.0 * (busy1 + busy2) / ((gui1 + gui2) / 8 * 1024)
    assert row[-3] == "2" and row[-2] == "2.0" and abs(float(row[-1]) - expect) < 0.05
