"""GPU: the error paths leave the library usable. Injected faults
(IQP_FAULT=launch / alloc) fail before any device work and later calls give
the same results as before; a corrupt tuning cache (IQP_TUNE_CACHE) is
skipped line by line: valid lines for the plan's shapes are used, anything
else leaves the default configuration, and results are unchanged."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest
import torch

import workloads as W
from paper_2501_04776_amd import api
from tests.gpu_util import DevWorkload

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _problems(dws):
    return [(api.Circuit(d.n, d.gens, d.theta), d.ops, d.samples) for d in dws]


def test_injected_faults_leave_the_library_usable(monkeypatch):
    w = W.small_random(31, 70, 900, 130, 700)
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    want = api.iqp_expval(circ, dw.ops, dw.samples, "split_bf16")[0].clone()
    monkeypatch.setenv("IQP_FAULT", "launch")
    with pytest.raises(RuntimeError, match="injected fault"):
        api.iqp_expval(circ, dw.ops, dw.samples, "split_bf16")
    monkeypatch.setenv("IQP_FAULT", "alloc")
    with pytest.raises(RuntimeError, match="injected fault"):
        api.BatchPlan(_problems([dw]), "split_bf16")
    monkeypatch.delenv("IQP_FAULT")
    got = api.iqp_expval(circ, dw.ops, dw.samples, "split_bf16")[0]
    plan = api.BatchPlan(_problems([dw]), "split_bf16")
    plan.expval()
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert np.abs(plan.means[0].cpu().numpy() - want.cpu().numpy()).max() < 1e-6
    plan.close()


# Runs in a fresh process: the cache file is read once per process.
_CHILD = textwrap.dedent("""
    import sys, json
    sys.path.insert(0, %r)
    import numpy as np, torch
    import workloads as W
    from paper_2501_04776_amd import api
    from tests.gpu_util import DevWorkload
    ws = [W.small_random(41 + i, 70 + 20 * i, 800, 90, 600) for i in range(2)]
    dws = [DevWorkload(w) for w in ws]
    plan = api.BatchPlan([(api.Circuit(d.n, d.gens, d.theta), d.ops, d.samples) for d in dws],
                         "split_bf16")
    plan.expval()
    torch.cuda.synchronize()
    print(json.dumps({"cfg": plan.config(),
                      "means": [m.cpu().numpy().tolist() for m in plan.means]}))
""") % ROOT


def _child(cache):
    env = dict(os.environ, IQP_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", _CHILD], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    import json
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_corrupt_tuning_cache_is_skipped(tmp_path):
    ref = _child(tmp_path / "absent")  # no file: the default configuration
    assert ref["cfg"]["tuned"] is False
    # the key of these shapes, as the plan writes it: precision, then
    # n,m,l,s of every problem
    key = "prec1:70,800,90,600;90,800,90,600;"
    bad = tmp_path / "bad"
    bad.write_bytes(b"\n".join([
        b"garbage without fields",
        b"\x00\xff\xfe binary \x01",
        key.encode() + b" 4 4",                       # too few fields
        key.encode() + b" 7 7 0 2 2",                 # no such tile
        key.encode() + b" 4 4 9 2 2",                 # no such split mode
        key.encode() + b" -4 4 0 2 2",
        b"prec1:1,2,3,4; 2 2 0 2 2",                  # valid line, other shapes
        b"x" * 100000,                                 # one very long line
        key.encode(),                                  # key alone
    ]) + b"\n")
    got = _child(bad)
    assert got["cfg"]["tuned"] is False
    assert got["means"] == ref["means"]
    # a valid line for these shapes among the junk is used
    good = tmp_path / "good"
    good.write_bytes(bad.read_bytes() + key.encode() + b" 2 2 1 2 4\n")
    got = _child(good)
    assert got["cfg"]["tuned"] is True
    assert tuple(got["cfg"]["fwd_tile"]) == (2, 2) and got["cfg"]["fwd_split"] == 1
    assert tuple(got["cfg"]["bwd_tile"]) == (2, 4)
    # another tile order sums the gate words in another order: results agree
    # to rounding
    assert np.abs(np.array(got["means"][0]) - np.array(ref["means"][0])).max() < 1e-4
