"""The committed HBM counters (profiles/hbm_traffic.json) belong to the current kernel
source: bench.py reports measured traffic only for the source the counters were taken
on, so a kernel change without new counters would leave the headline line without its
measured traffic. CPU only."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_headline_counters_match_the_kernel_source():
    for workload, kernel in (("pareto_100k", "resident"), ("pareto_100k", "centrality"),
                             ("pareto_100k:plain", "resident"), ("sbm_10k", "resident"),
                             ("smallcut_100k", "resident")):
        t = bench.measured_traffic(workload, kernel)
        assert t is not None and t > 0, (workload, kernel)
