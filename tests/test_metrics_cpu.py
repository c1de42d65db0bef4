"""The JSON-lines metrics records, on hand-made solve results (no GPU)."""
import json

import numpy as np
import torch

import paper_2403_17018_amd as P
from paper_2403_17018_amd.metrics import BYTES_PER_UNIT, MetricsLog, batch_record, kernel_classes


def _result(stats, status):
    return P.SolveResult(c_T=None, p_T=None, qoi=torch.zeros(len(status), dtype=torch.float64),
                         status=torch.tensor(status, dtype=torch.int32),
                         stats=torch.tensor(stats, dtype=torch.float64), nfailed=int(np.count_nonzero(status)))


def test_batch_record_histograms_statuses_and_throughput():
    g = P.grid(32, 16, 10)
    # Newton iterations over 10 steps: 10, 15, 20 -> 1.0, 1.5, 2.0 per step; BiCGStab: 10, 30, 20
    r = _result([[10, 10, 1e-9, 2e-9], [15, 30, 3e-9, 1e-9], [20, 20, 0.0, 5e-9]], [0, 4, 0])
    rec = batch_record("t", g, r, seconds=0.5)
    h = rec["newton_per_step"]
    assert h["edges"][0] == 1.0 and h["edges"][-1] == 2.25 and sum(h["counts"]) == 3
    assert h["counts"] == [1, 0, 1, 0, 1] and h["mean"] == 1.5
    k = rec["krylov_per_newton"]
    assert (k["min"], k["max"]) == (1.0, 2.0) and sum(k["counts"]) == 3
    assert rec["status_counts"] == {"0": 2, "4": 1} and rec["failed"] == 1
    assert rec["max_fluid_defect"] == 3e-9 and rec["max_salt_defect"] == 5e-9
    assert rec["sample_timesteps_per_s"] == 3 * 10 / 0.5
    json.dumps(rec)   # serialisable as is


def test_kernel_classes_bandwidth():
    # 10 launches of the FP64 smoother over 1e6 cell-samples each in 1 ms total
    prof = {"gs": (10, 10_000_000, 1.0), "band_factor": (2, 64, 0.1), "spmv": (0, 0, 0.0)}
    kc = kernel_classes(prof, 64)
    assert "spmv" not in kc and "gbs" not in kc["band_factor"]
    want = 10_000_000 * BYTES_PER_UNIT[64]["gs"] / 1e-3 / 1e9
    assert abs(kc["gs"]["gbs"] - round(want, 2)) < 1e-9 and kc["gs"]["avg_launch_us"] == 100.0


def test_metrics_log_appends_lines(tmp_path):
    path = tmp_path / "m.jsonl"
    with MetricsLog(str(path)) as log:
        log.write({"a": 1})
    with MetricsLog(str(path)) as log:
        log.write({"b": 2})
    assert [json.loads(x) for x in path.read_text().splitlines()] == [{"a": 1}, {"b": 2}]
