"""Host-side tools around the path (CPU only): the counter-run summariser
and the benchmark's traffic lookup, the autotuner's cache mapping, the
oracle sample behind the CPU baseline, and the batch workload generator."""

import csv
import json
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2510_24968_amd import autotune, prof_traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, values) in enumerate(rows):
            for v in values:          # one row per counter instance, summed by dispatch
                w.writerow({k: 0 for k in FIELDS} | {
                    "Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                    "Counter_Value": v, "Start_Timestamp": 1000 * i,
                    "End_Timestamp": 1000 * i + 2_000_000})


def test_traffic_summary_scales_by_the_copy_and_skips_stored_blocks(tmp_path):
    lane = "void fsim::k_eri_lane_ko<1, 1, 1, 0, double, false, 3, 3>(fsim::EriArgs)"
    store = "void fsim::k_eri_lane<1, 1, 1, 0, double, true, 3, 3>(fsim::EriArgs)"
    f32 = "void fsim::k_eri_lane<2, 1, 1, 1, float, false, 6, 2>(fsim::EriArgs)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = [(copy, [262144.0, 262144.0]), (store, [5.0]), (lane, [100.0, 300.0]), (f32, [8.0])]
    write = [(copy, [1048576.0]), (store, [7.0]), (lane, [50.0]), (f32, [2.0])]
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    s = prof_traffic.summarise(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert s["fetch_factor"] == pytest.approx(2.0)      # 1 GiB copy read as 512 MiB
    assert s["write_factor"] == pytest.approx(1.0)
    k = s["kernels"]
    assert set(k) == {"(pp|ps)", "(dp|pp) f32"}          # the stored-block launch is not Fock work
    assert k["(pp|ps)"]["bytes_per_launch"] == pytest.approx((400.0 * 2.0 + 50.0) * 1024)
    assert k["(pp|ps)"]["kernel"] == "k_eri_lane_ko<1, 1, 1, 0, double, false, 3, 3>"


def test_bench_traffic_needs_matching_sources(monkeypatch):
    import bench
    path = os.path.join(ROOT, "profiles", "k_eri_water64_fp64_traffic.md")
    blob = json.loads(open(path).read().split("```json")[1].split("```")[0])
    # the summary's figures are used only for the kernel sources it was taken on
    monkeypatch.setattr(prof_traffic, "source_digest", lambda: blob["source_digest"])
    rec = bench.kernel_traffic("water64", {"cls": "(pp|ps)"})
    assert rec == blob["kernels"]["(pp|ps)"]["bytes_per_launch"]
    assert bench.kernel_traffic("water64", {"cls": "(xx|yy)"}) is None
    assert bench.kernel_traffic("no_such_workload", {"cls": "(pp|ps)"}) is None
    monkeypatch.setattr(prof_traffic, "source_digest", lambda: "0" * 16)
    assert bench.kernel_traffic("water64", {"cls": "(pp|ps)"}) is None


def test_sq_summary_counts_fp64_flops_per_lane(tmp_path):
    """64 flops per FP64 ADD/MUL/TRANS wave instruction, 128 per FMA, 512
    per FP64 MFMA MOPS, over the dispatch's duration; the longest launch of
    a class is kept (the FP64 build's full list)."""
    from paper_2510_24968_amd import prof_sq
    seg = "void fsim::k_eri_lane_ko<1, 1, 1, 0, double, false, 3, 3, true>(fsim::EriArgs)"
    sq = tmp_path / "sq.csv"
    mix = tmp_path / "mix.csv"
    with open(sq, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for cname, v in (("SQ_WAVE_CYCLES", 1000.0), ("SQ_WAIT_ANY", 250.0),
                         ("SQ_ACTIVE_INST_VALU", 500.0)):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": 1, "Kernel_Name": seg,
                                                 "Counter_Name": cname, "Counter_Value": v,
                                                 "Start_Timestamp": 0, "End_Timestamp": 2_000_000})
    with open(mix, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, ns in ((1, 2_000_000), (2, 1_000_000)):     # a shorter second launch is ignored
            for cname, v in (("SQ_INSTS_VALU_FMA_F64", 1e6), ("SQ_INSTS_VALU_ADD_F64", 2e6),
                             ("SQ_INSTS_VALU_MFMA_MOPS_F64", 1e3)):
                w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": d, "Kernel_Name": seg,
                                                     "Counter_Name": cname, "Counter_Value": v,
                                                     "Start_Timestamp": 0, "End_Timestamp": ns})
    r = prof_sq.summarise(str(sq), str(mix))["(pp|ps)"]
    flops = 64 * (2e6 + 2 * 1e6) + 512 * 1e3
    assert r["fp64_flops_issued"] == pytest.approx(flops)
    assert r["fp64_tflops_issued"] == pytest.approx(flops / 2e-3 / 1e12)
    assert r["wait"] == pytest.approx(0.25) and r["valu_busy"] == pytest.approx(0.5)


def test_bench_counters_need_matching_sources(monkeypatch):
    import bench
    path = os.path.join(ROOT, "profiles", "k_eri_water64_fp64_sq_counters.md")
    blob = json.loads(open(path).read().split("```json")[1].split("```")[0])
    monkeypatch.setattr(prof_traffic, "source_digest", lambda: blob["source_digest"])
    rec = bench.kernel_counters("water64", {"cls": "(pp|ps)"})
    assert rec["fp64_tflops_issued"] == blob["kernels"]["(pp|ps)"]["fp64_tflops_issued"]
    monkeypatch.setattr(prof_traffic, "source_digest", lambda: "0" * 16)
    assert bench.kernel_counters("water64", {"cls": "(pp|ps)"}) is None


class _FakeCtx:
    def __init__(self, recs):
        self.recs = recs
        self.set = None

    def get_tuning(self):
        return self.recs

    def set_tuning(self, recs):
        self.set = recs


def test_autotune_cache_keys_and_apply():
    recs = [dict(cls="(pp|ps)", bra_class=2, ket_class=1, fp32=0, variant=1, waves_per_block=4,
                 kbra=9, kket=9, ms=0.0),
            dict(cls="(pp|ps)", bra_class=2, ket_class=1, fp32=1, variant=1, waves_per_block=4,
                 kbra=9, kket=9, ms=0.0),
            dict(cls="(ss|ss)", bra_class=0, ket_class=0, fp32=0, variant=1, waves_per_block=4,
                 kbra=1, kket=1, ms=0.0)]
    assert autotune.cache_key(recs[0]) == "(pp|ps)|fp64|K9x9"
    assert autotune.cache_key(recs[1]) == "(pp|ps)|fp32|K9x9"
    table = {"(pp|ps)|fp64|K9x9": dict(variant=4, waves_per_block=2, ms=1.5),
             "(ss|ss)|fp64|K9x9": dict(variant=0, waves_per_block=1, ms=0.1)}   # other K: no hit
    ctx = _FakeCtx(recs)
    assert autotune.apply(ctx, table) == 1
    assert ctx.set == [dict(bra_class=2, ket_class=1, fp32=0, variant=4, waves_per_block=2,
                            seg_tiles=0, ms=1.5)]


def test_committed_tuning_caches_are_well_formed():
    for name in ("water64_mi355x.json", "ch1024_mi355x.json"):
        entries = autotune.load(os.path.join(ROOT, "paper_2510_24968_amd", "tuning", name))
        assert entries
        for key, e in entries.items():
            assert key == autotune.cache_key(e)
            assert 0 <= e["variant"] < 7 and e["waves_per_block"] in (1, 2, 4, 8)
            assert e.get("seg_tiles", 0) in (0, 16, 32, 64, 128, 256, 512)


def test_cpu_baseline_samples_kept_quartets():
    """The baseline's oracle sample only holds Schwarz-kept canonical
    quartets, and its rate is quartets over oracle time."""
    import bench
    import torch
    basis = synth.water_cluster(2, 3)
    B = oracle.Basis(basis)
    S, T, V = B.one_electron()
    X = oracle.orthogonalizer(S)
    D, _, _ = oracle.density_from_fock(T + V, X, B.nelec // 2)
    w = {"tau": 1e-9}
    res = bench.cpu_baseline(basis, w, torch.tensor(D), target_s=0.3)
    assert res["kind"] == "oracle" and res["value"] > 0 and res["cores"] >= 1
    n = int(res["sample"].split()[0])
    assert n >= 20_000


def test_ch_molecules_respect_their_construction():
    for seed in range(4_000_000, 4_000_040):
        b = synth.ch_molecule(seed)
        n = len(b["types"])
        assert 2 <= n <= 24
        assert b["nelec"] % 2 == 0
        xyz = np.asarray(b["xyz"])
        d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1) + np.eye(n) * 1e9
        assert d.min() >= 1.8 - 1e-12
        steps = np.linalg.norm(np.diff(xyz, axis=0), axis=1)
        assert np.all((steps >= 2.0 - 1e-12) & (steps <= 2.9 + 1e-12))
        nbf = synth.nbf_of(b)
        assert nbf == sum(8 if t == "C" else 4 for t in b["types"])


def test_product_path_fails_loudly_without_gpu_or_library(monkeypatch):
    """No CPU fallback: without a GPU the context refuses to start, and
    without the built library the binding raises instead of substituting
    anything."""
    import torch
    from paper_2510_24968_amd import fsim
    if not torch.cuda.is_available():
        with pytest.raises(fsim.FsimError, match="GPU"):
            fsim.Context(synth.h_chain(2, 1.4))
        with pytest.raises(fsim.FsimError, match="GPU"):
            fsim.Batch([synth.h_chain(2, 1.4)])
    monkeypatch.setattr(fsim, "_lib", None)
    monkeypatch.setattr(fsim, "LIBPATH", "/nonexistent/libfsim.so")
    with pytest.raises(fsim.FsimError, match="not built"):
        fsim.lib()
