"""The committed rocprofv3 summaries against the sources they describe (no GPU).

* Every summary under profiles/ gives the command that produced it, and that
  command runs committed files only (bench.py, no scratch scripts).
* The HBM counter summaries of the benchmark's default workload (the k-mesh
  B and C products, workload 5) and of the molecular default (the fused
  kernel, workload 2) were taken on the current kernel sources: bench.py
  reports their traffic (`roofline.traffic`) only while the recorded source
  hash matches, so an edit of those kernels without new counters fails here.
"""
import glob
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_summary_names_its_command(path):
    text = open(path).read()
    cmds = re.findall(r"rocprofv3 [^\n]*", text)
    assert cmds, "no rocprofv3 command"
    for c in cmds:
        if " -- " not in c:
            continue
        prog = c.split(" -- ", 1)[1]
        assert prog.startswith("python3 bench.py"), prog
        assert "_work" not in c


@pytest.mark.parametrize("workload,precision,kind", [(5, "bf16x3", "solid"), (2, "fp32", "bare")])
def test_default_workload_counters_match_sources(workload, precision, kind):
    traffic = bench.read_traffic(workload, precision, kind)
    assert traffic is not None and traffic > 0
