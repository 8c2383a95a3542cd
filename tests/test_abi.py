"""CPU checks of the C ABI library: it loads and exports every entry point
declared in include/fftg.h (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fftg.h")).read()
    return re.findall(r"^(?:fftg_status|const char\*)\s+(\w+)\(", src, re.M)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fftg_create", "fftg_destroy", "fftg_last_error", "fftg_solve",
              "helmholtz_solve", "staggered_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_04770_amd import binding
    if not os.path.exists(binding.lib_path()):
        from paper_2103_04770_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(binding.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_create_rejects_bad_grids_without_touching_the_gpu():
    """Validation happens before any device call."""
    from paper_2103_04770_amd import binding
    lib = binding.load_library()
    bad = [(3, (10, 8, 8)), (3, (8, 7, 8)), (4, (8, 8, 8)), (3, (9, 8, 8)), (2, (512 * 3, 8, 1))]
    codes = []
    for ndim, n in bad:
        g = binding.Grid(ndim, (ctypes.c_int * 3)(*n), 1.0, 0, 0)
        h = ctypes.c_void_p()
        codes.append(lib.fftg_create(ctypes.byref(g), None, ctypes.byref(h)))
        assert not h.value
        assert lib.fftg_last_error(None)
    assert codes == [-2, -2, -1, -2, -2]


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes mirrors of the public structs have the sizes and
    field offsets the C compiler gives the header's declarations."""
    import shutil
    import subprocess
    from paper_2103_04770_amd import binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    checks = {
        "fftg_phase": (binding.Phase, ["model", "E", "dfield", "dmax", "ell", "n_hard", "q1",
                                       "sN", "fu"]),
        "fftg_macro": (binding.Macro, ["mask", "E", "S"]),
        "fftg_stats": (binding.Stats, ["newton_iters", "relres", "err", "t_ms",
                                        "inner_converged"]),
        "fftg_drive_opts": (binding.DriveOpts, None),
        "fftg_drive_record": (binding.DriveRecord, None),
        "fftg_batch_item": (binding.BatchItem, None),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fftg.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in fields or []:
            cf = {"n_hard": "n_hard"}.get(f, f)
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, cf))
    lines.append("return 0; }")
    src = tmp_path / "sz.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for cname, (cls, fields) in checks.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for f in fields or []:
            assert int(out["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_run_config_round_trip_and_byte_model():
    """The run configuration survives JSON, rejects unknown keys, and the
    per-iteration byte model equals the fused-pass counts at 128^3."""
    from paper_2103_04770_amd.run import RunConfig, bytes_per_iteration
    cfg = RunConfig(workload="spheres64_20", e11_end=0.02, precision="fp32_refined",
                    table_overrides=[{"dC": 0.001}], log="x.jsonl")
    back = RunConfig.from_json(cfg.to_json())
    assert back == cfg
    with pytest.raises(ValueError):
        RunConfig.from_json('{"workload": "spheres64_20", "bogus": 1}')
    Ns, N = 128 * 128 * 65, 128 ** 3
    g, h = bytes_per_iteration((128, 128, 128), "fp64")
    assert g == 18 * 6 * Ns * 16 + 8 * N * 8
    # x pass 6, y passes 5 + 5, outer passes 7 + 4 (two fields), residual 3
    assert h == (6 + 10 + 7 + 4 + 3) * Ns * 16 + N * 8
    g2, _ = bytes_per_iteration((32, 32), "fp32_refined")
    assert g2 == 14 * 3 * 32 * 17 * 8 + 8 * 32 * 32 * 4


def test_profiling_summaries_on_synthetic_csv(tmp_path):
    """Host logic of the rocprofv3 summaries: kernel classes (the split
    Helmholtz y pass by direction), counter calibration against the device
    copy and the per-pass HBM rate, on small hand-made CSV files."""
    from paper_2103_04770_amd import profiling as pr
    assert pr.classify("void fftg::k_h_y_split<double, true, 128>") == ("fp64", "helmholtz_y_fwd")
    assert pr.classify("void fftg::k_h_y_split<float, false, 64>") == ("fp32", "helmholtz_y_inv")
    assert pr.classify("void fftg::k_gal_dir_inv<double, 128, 0>") == ("fp64",
                                                                       "galerkin_outer_dir_inv")
    assert pr.classify("fftg::k_stream_copy") is None
    k = "void fftg::k_gal_resid<double, 6>"
    trace = tmp_path / "trace.csv"
    q = '"%s"' % k                       # rocprofv3 quotes the names (they hold commas)
    trace.write_text("Kernel_Name,Start_Timestamp,End_Timestamp\n"
                     "%s,0,50000\n%s,100000,150000\n%s,200000,201000\n" % (q, q, q))
    for name, counter, copy_kib, kib in (("f", "FETCH_SIZE", 512.0, 150.0),
                                         ("w", "WRITE_SIZE", 1024.0, 100.0)):
        d = tmp_path / name
        d.mkdir()
        (d / "run_counter_collection.csv").write_text(
            "Kernel_Name,Counter_Name,Counter_Value\n"
            "__amd_rocclr_copyBuffer,%s,%f\n%s,%s,%f\n%s,%s,%f\n" % (
                counter, copy_kib, q, counter, kib, q, counter, kib))
    text = pr.rates(str(trace), str(tmp_path / "f"), str(tmp_path / "w"), 1, "t", "c")
    row = [l for l in text.splitlines() if l.startswith(k)][0].split()
    # two full launches of 50 us (the 1 us one is left out); fetch scaled x2
    # (1 MiB copy read as 512 KiB), write x1: (300 + 100) KiB per launch
    full, us, mb, gbs = int(row[-5]), float(row[-4]), float(row[-3]), float(row[-2])
    assert full == 2 and us == pytest.approx(50.0)
    assert mb == pytest.approx(400 * 1024 / 1e6, abs=0.05)
    assert gbs == pytest.approx(400 * 1024 / 50e-6 / 1e9, abs=0.5)   # printed to 1 GB/s
    # the same launches in both runs: paired one by one (a lockstep launch
    # with fewer live systems moves fewer bytes in less time)
    k2 = "void fftg::k_h_div_fwd<double, 128, 3, true>"
    q2 = '"%s"' % k2
    trace.write_text("Kernel_Name,Start_Timestamp,End_Timestamp\n"
                     "%s,300000,360000\n%s,0,50000\n%s,100000,110000\n" % (q2, q2, q2))
    for name, counter, copy_kib in (("f", "FETCH_SIZE", 512.0), ("w", "WRITE_SIZE", 1024.0)):
        vals = (100.0, 20.0, 100.0) if counter == "FETCH_SIZE" else (200.0, 40.0, 200.0)
        (tmp_path / name / "run_counter_collection.csv").write_text(
            "Kernel_Name,Counter_Name,Counter_Value,Dispatch_Id\n"
            "__amd_rocclr_copyBuffer,%s,%f,1\n%s,%s,%f,2\n%s,%s,%f,3\n%s,%s,%f,4\n" % (
                counter, copy_kib, q2, counter, vals[0], q2, counter, vals[1], q2, counter,
                vals[2]))
    text = pr.rates(str(trace), str(tmp_path / "f"), str(tmp_path / "w"), 1, "t", "c")
    row = [l for l in text.splitlines() if l.startswith(k2)][0]
    assert "true> *" in row
    f = row.split()
    # launches in start order: 50, 10, 60 us with 400, 80, 400 KiB: the
    # first and last are full, 800 KiB in 110 us
    assert int(f[-5]) == 2 and float(f[-4]) == pytest.approx(55.0)
    assert float(f[-2]) == pytest.approx(800 * 1024 / 110e-6 / 1e9, abs=0.5)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
