"""Host logic of the benchmark's counter summaries (CPU only): the HBM bytes
per walk from FETCH_SIZE / WRITE_SIZE scaled by a copy's calibration,
and the wave instructions per unit of work from SQ_INSTS_VALU / SQ_INSTS_SALU,
on small hand-made counter files."""
import csv
import json
import subprocess
import sys
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(("Kernel_Name", "Counter_Name", "Counter_Value"), r)))


def _bench(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       cwd=ROOT)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_summarize_counters_scales_by_the_copy(tmp_path):
    f, w, cf, cw = (str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    # two walks (each opened by a first tile generation), a later generation,
    # a tail walk and its prefix kernel: 1000 + 250 + 500 + 2500 + 750 KiB fetched
    gen0, gen = "tile_walk_kernel<true, true, false>(P)", "tile_walk_kernel<true, false, false>(P)"
    _csv(f, [(gen0, "FETCH_SIZE", 1000), (gen, "FETCH_SIZE", 250), ("tail_prefix_kernel", "FETCH_SIZE", 500),
             ("tail_walk_kernel<true, false>", "FETCH_SIZE", 2500), (gen0, "FETCH_SIZE", 750),
             ("pack_kernel", "FETCH_SIZE", 99999)])
    _csv(w, [(gen0, "WRITE_SIZE", 10), ("tail_walk_kernel<true, false>", "WRITE_SIZE", 30),
             (gen0, "WRITE_SIZE", 0)])
    # a 1 MiB copy whose fetch counter reads half of what it moves
    _csv(cf, [("neg_kernel", "FETCH_SIZE", 512)])
    _csv(cw, [("neg_kernel", "WRITE_SIZE", 1024)])
    out = str(tmp_path / "traffic.json")
    r = _bench("--summarize-counters", f, w, cf, cw, "--calibration-mib", "1", "--traffic", out)
    assert r["fetch_scale"] == pytest.approx(2.0) and r["write_scale"] == pytest.approx(1.0)
    assert r["counted"]["fetch"] == {"launches": 4, "walks": 2}
    assert r["fetch_bytes_per_walk"] == pytest.approx(2.0 * 5000 * 1024 / 2)
    assert r["write_bytes_per_walk"] == pytest.approx(40 * 1024 / 2)
    assert json.load(open(out))["bytes_per_walk"] == pytest.approx(r["bytes_per_walk"])


def test_summarize_valu_divides_by_the_profiled_work(tmp_path):
    c = str(tmp_path / "c.csv")
    _csv(c, [("tile_walk_kernel<true>", "SQ_INSTS_VALU", 6e9), ("tail_walk_kernel", "SQ_INSTS_VALU", 3e9),
             ("tile_walk_kernel<true>", "SQ_INSTS_SALU", 1e9), ("pack_kernel", "SQ_INSTS_VALU", 5e12)])
    log = str(tmp_path / "b.log")
    with open(log, "w") as fh:
        fh.write("noise\n" + json.dumps({"metric": "photon cell-crossings/s", "steps": 2, "warmup": 1,
                                         "config": {"workload": "w", "crossings_per_step": 1e8}}) + "\n")
    out = str(tmp_path / "v.json")
    r = _bench("--summarize-valu", c, log, out)
    assert r["valu_wave_instr_per_crossing"] == pytest.approx(9e9 / 3e8)
    assert r["salu_wave_instr_per_crossing"] == pytest.approx(1e9 / 3e8)
    assert r["config"] == "c3" and r["profile"] == "doppler"
    with open(log, "w") as fh:
        fh.write(json.dumps({"metric": "resonant scatterings/s", "steps": 1, "warmup": 0,
                             "config": {"workload": "s", "scatterings_per_step": 2e9, "photons": 64}}) + "\n")
    _csv(c, [("scatter_kernel<false, true>", "SQ_INSTS_VALU", 1e11), ("scatter_kernel<false, true>",
                                                                       "SQ_INSTS_SALU", 2e10)])
    r = _bench("--summarize-valu", c, log, out)
    assert r["valu_wave_instr_per_scattering"] == pytest.approx(50.0) and r["photons"] == 64


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    import bench
    a, b, c = (tmp_path / n for n in ("a.hip", "b.hip", "c.hip"))
    a.write_text("// header\nint f(int x) { return x + 1; }  /* done */\n")
    b.write_text("int f(int x)\n{\n    return x + 1;   // one more\n}\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash(["a.hip"]) == bench.source_hash(["b.hip"])
    assert bench.source_hash(["a.hip"]) != bench.source_hash(["c.hip"])
