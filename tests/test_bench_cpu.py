"""Host-side parts of bench.py (no GPU): the one-GPU contract, the roofline
object, the stored HBM byte counts and their source hash, and the schedule
file round trip."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_picks_the_dominant_stage_and_binding_peak():
    st = [{"name": "spread", "ms_total": 3.0, "ms_avg": 3.0, "bytes": 1e9, "flops": 1e12},
          {"name": "fft2", "ms_total": 4.0, "ms_avg": 4.0, "bytes": 4e9, "flops": 4e10}]
    r = bench.roofline(st, "f32", None)
    assert r["ms_avg"] == 4.0 and r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(4e9 / 4e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    st[1]["flops"] = 1e15   # now the flop rate binds
    r = bench.roofline(st, "f32", None)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"


def test_stored_traffic_only_for_its_sources_and_workload():
    """A stored HBM byte count is reported only while the sources it was
    measured on are unchanged (comments aside) and for its own workload."""
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["fft2"]
    st = [{"name": "fft2", "ms_total": 4.0, "ms_avg": 4.0, "bytes": 4e9, "flops": 4e10}]
    same = t["source_sha"] == bench._source_sha()
    got = bench.roofline(st, "f32", t["P"])["traffic"]
    assert got == (pytest.approx(t["bytes_per_launch"]) if same else None)
    assert bench.roofline(st, "f32", t["P"] + 2)["traffic"] is None


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    import shutil
    csrc = os.path.join(ROOT, "paper_1712_04732_amd", "csrc")
    fake = tmp_path / "paper_1712_04732_amd" / "csrc"
    shutil.copytree(csrc, fake)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench._source_sha()
    f = fake / "se_fft.hip"
    f.write_text("// a comment line\n" + f.read_text().replace("namespace se {", "namespace se {  // trailing"))
    assert bench._source_sha() == h0
    f.write_text(f.read_text().replace("namespace se {", "namespace se {   \n\n", 1))
    assert bench._source_sha() == h0        # trailing blanks and blank lines
    f.write_text(f.read_text() + "\nint extra_symbol;\n")
    assert bench._source_sha() != h0


def test_schedule_round_trip(tmp_path):
    from paper_1712_04732_amd import _lib as L
    ps = []
    for D, M in ((3, 32), (0, 48)):
        p = L.se_params()
        p.D, p.M = D, M
        p.tile3[0], p.tile3[1], p.tile3[2] = 16, 16, 8
        p.fft_cap, p.xcd_tiles, p.xcd_fft, p.spread_mode = 4096, 8, -1, 3
        ps.append(p)
    path = str(tmp_path / "s.json")
    bench._save_schedule(path, ps)
    qs = []
    for D, M in ((3, 32), (0, 48)):
        q = L.se_params()
        q.D, q.M = D, M
        qs.append(q)
    assert bench._load_schedule(path, qs)
    for p, q in zip(ps, qs):
        assert list(q.tile3) == list(p.tile3) and q.fft_cap == p.fft_cap
        assert (q.xcd_tiles, q.xcd_fft, q.spread_mode) == (p.xcd_tiles, p.xcd_fft, p.spread_mode)
    qs[1].M = 50   # a schedule for other systems is not applied
    assert not bench._load_schedule(path, qs)


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_pair_count_matches_brute_force(D):
    import numpy as np
    rng = np.random.default_rng(5 + D)
    N, L, rc = 400, 1.0, 0.23
    x = rng.random((N, 3)) * L
    d = x[:, None, :] - x[None, :, :]
    for k in range(D):                  # nearest image in the periodic directions (rc < L/2)
        d[..., k] -= L * np.round(d[..., k] / L)
    r = np.sqrt((d * d).sum(-1))
    brute = (np.count_nonzero(r < rc) - N) / N
    assert abs(bench.pairs_within(D, L, rc, x, n_sample=N) - brute) < 1e-12


def test_real_space_traffic_only_for_matching_sources_and_workload():
    """The real-space bench line reports stored HBM bytes only when they were
    taken on the current sources (comment-free hash) and the same workload."""
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    ent = t.get("rs_pairs")
    if ent is None:
        pytest.skip("no stored real-space byte count")
    if ent["source_sha"] == bench._source_sha(bench.RS_SOURCES):
        assert bench._rs_traffic(ent["workload"]) == ent["bytes_per_launch"]
    else:
        assert bench._rs_traffic(ent["workload"]) is None
    assert bench._rs_traffic("no such workload") is None


def _pmc_csv(path, counter, rows):
    hdr = ("Correlation_Id,Dispatch_Id,Agent_Id,Queue_Id,Process_Id,Thread_Id,Grid_Size,Kernel_Id,Kernel_Name,"
           "Workgroup_Size,LDS_Block_Size,Scratch_Size,VGPR_Count,Accum_VGPR_Count,SGPR_Count,Counter_Name,"
           "Counter_Value,Start_Timestamp,End_Timestamp")
    with open(path, "w") as f:
        f.write(hdr + "\n")
        for i, (k, v) in enumerate(rows):
            f.write(f'{i},{i},"Agent 1",1,1,1,256,{i},"{k}",256,0,0,8,0,32,"{counter}",{v},0,1\n')


def test_traffic_from_counter_csvs(tmp_path, monkeypatch):
    """--traffic-from: per-launch means of FETCH_SIZE and WRITE_SIZE (KiB) by
    kernel, scaled so that the calibration copy reads and writes 256 MiB;
    other kernels and the FP64 instances are ignored."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_source_sha", lambda files=None: "abc")
    k = "void se::batch_fft_kernel<float, 4, unsigned int>(se::SysDesc const*, int)"
    k64 = "void se::batch_fft_kernel<double, 4, unsigned int>(se::SysDesc const*, int)"
    g = "void se::batch_stage_kernel<float, 10, 13>(se::SysDesc const*, int)"
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", [(k, 1000.0), (k, 3000.0), (k64, 9e9), (g, 500.0), ("other", 1.0)])
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(k, 4000.0), (k, 4000.0), (g, 50.0)])
    _pmc_csv(tmp_path / "cf.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 131072.0)] * 5)
    _pmc_csv(tmp_path / "cw.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0)] * 5)
    bench.main_traffic_from([str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")])
    out = json.load(open(prof / "traffic.json"))
    assert set(out) == {"fft2", "gather"}
    e = out["fft2"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert e["write_bytes"] == pytest.approx(4000.0 * 1024)
    assert e["bytes_per_launch"] == pytest.approx(e["fetch_bytes"] + e["write_bytes"])
    assert e["source_sha"] == "abc" and e["P"] == 10 and e["workload"] == "C5_batch"
