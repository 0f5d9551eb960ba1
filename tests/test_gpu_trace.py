"""roctx ranges and marks of the library, as rocprofv3 --marker-trace records them.

A child process runs one plain registration, one batch and one served request
under rocprofv3; its marker trace must hold the host-side phases the library
names (dses.registration with dses.prepare and dses.sweep_select inside it,
dses.batch, dses.target_create, dses.slice_launch, dses.request_done).
"""
import csv
import glob
import os
import shutil
import subprocess
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = """
import sys
sys.path.insert(0, {root!r})
from paper_2502_00115_amd import dses, synth
p = synth.make_c1(0)
dses.register(p.src, p.tgt, p.rotations, p.eps)
dses.register_batch([dict(src=p.src, tgt=p.tgt, rotations=p.rotations, eps=p.eps)],
                    use_graph=False)
t, r = dses.Target(p.tgt), dses.RotationSet(p.rotations)
srv = dses.Server(memory_budget=64 << 20, max_inflight=4)
srv.wait(srv.submit(t, r, p.src, p.eps), timeout_ms=60000)
srv.close()
print("child done", flush=True)
"""


def test_host_phases_are_roctx_ranges(tmp_path):
    rp = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(rp):
        pytest.skip("rocprofv3 not installed")
    script = tmp_path / "child.py"
    script.write_text(CHILD.format(root=ROOT))
    env = dict(os.environ, TMPDIR=str(tmp_path))
    out = tmp_path / "trace"
    r = subprocess.run([rp, "--marker-trace", "--output-format", "csv", "-d", str(out), "-o",
                        "run", "--", sys.executable, str(script)],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=300)
    assert "child done" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    files = glob.glob(str(out / "**" / "*marker_api_trace.csv"), recursive=True)
    assert files, r.stderr[-2000:]
    names = set()
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                names.update(v for v in row.values() if isinstance(v, str))
    want = {"dses.registration", "dses.prepare", "dses.sweep_select", "dses.batch",
            "dses.target_create", "dses.slice_launch", "dses.request_done"}
    assert want <= names, sorted(names)
