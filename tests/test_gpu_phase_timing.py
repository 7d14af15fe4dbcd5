"""The profiling build of the library (phase stamps in the persistent
kernel): its results equal the oracle's, every task is counted once per
launch and every phase takes time; the regular library refuses the call."""

import json
import os
import subprocess
import sys

import pytest

import synth
import paper_1610_04124_amd as P
from paper_1610_04124_amd import binding as B
from gpu_helpers import announce, device

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import oracle, synth, paper_1610_04124_amd as P
from gpu_helpers import assert_frames_equal
params = synth.make_params()
h = P.Stixels(params)
frames = [synth.generate_frame(synth.SceneSpec(seed=s)) for s in (3, 4)]
dev = torch.device("cuda", 0)
d = [torch.from_numpy(f).to(dev) for f in frames]
outs = [h.new_output(1024, 440) for _ in d]
b = P.Batch(2, 2 * 204, 440, 128)
b.compute(list(zip([h, h], d, outs)))
b.compute(list(zip([h, h], d, outs)))
torch.cuda.synchronize()
for f, o in zip(frames, outs):
    assert_frames_equal(o.to_host(), oracle.frame(params, f), "phase-timing build")
print(json.dumps(b.phase_cycles()))
"""


def test_phase_timing_build_counts_every_task_and_matches_oracle():
    if not os.path.exists(B.PHASES_LIB_PATH):
        pytest.skip("libstixels_phases.so not built (python -m paper_1610_04124_amd.build "
                    "--phase-timing)")
    announce("phase-timing library, 2 frames 1024x440, two launches (child process)")
    env = dict(os.environ, STIXELS_PHASE_TIMING="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True,
                       text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-3000:]
    c = json.loads(r.stdout.strip().splitlines()[-1])
    assert c["tasks"] == 2 * 2 * 204
    for k in ("reduce", "prefix_scans", "object_table", "recurrence", "backtracking"):
        assert c[k] > 0, (k, c)
    assert c["recurrence"] > c["reduce"]
    busy = sum(c[k] for k in ("reduce", "prefix_scans", "object_table", "recurrence",
                              "backtracking"))
    assert busy <= c["workgroup_lifetime"]


def test_regular_library_refuses_phase_cycles():
    announce("phase cycles from the regular library")
    device()
    if os.environ.get("STIXELS_PHASE_TIMING") == "1":
        pytest.skip("this process loaded the phase-timing library")
    b = P.Batch(1, 204, 440, 128)
    with pytest.raises(B.StixelsError) as e:
        b.phase_cycles()
    assert e.value.code == B.E_INVALID_ARG
