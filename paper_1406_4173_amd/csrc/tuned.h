// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from
// timings on one MI355X; edit by re-running it, not by hand.
//
// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to
// tuned_mid_range with 512, larger ones with 1024. A group holds
// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes
// with more than n >> tuned_dense_shift bits scans the range instead.
// Dijkstra_SK groups (forward only, integer results, so any launch shape gives the same
// bits) have their own thresholds, tuned_dsk_small_range and tuned_dsk_mid_range, and
// hold max(8, tuned_dsk_group_work / w) of their part's sources, at most 64, where w is
// the part's nodes plus arcs (0: always 64). The count depends on the part alone, so a
// part is split the same way in every build that holds it.
//
// Timings of the sweep (ms, best of 2 after a warm-up run):
//   256 to 2000 512 to 5000 div  256: sbm_10k plain   10.74  sbm_10k pp   11.36  planted_1k plain    0.50  planted_1k pp    0.84  batch_256 plain    7.73  batch_256 pp   18.97
//   256 to 1500 512 to 4000 div  256: sbm_10k plain   10.73  sbm_10k pp   11.36  planted_1k plain    0.50  planted_1k pp    0.85  batch_256 plain    8.71  batch_256 pp   20.18
//   256 to 2000 512 to 6000 div  256: sbm_10k plain   10.73  sbm_10k pp   11.27  planted_1k plain    0.50  planted_1k pp    0.84  batch_256 plain    7.76  batch_256 pp   18.92
//   256 to 2500 512 to 5000 div  256: sbm_10k plain   10.69  sbm_10k pp   11.32  planted_1k plain    0.50  planted_1k pp    0.85  batch_256 plain    7.95  batch_256 pp   19.23
//   Dijkstra_SK 256 to 2000 512 to 5000 work      0: pareto_100k pp   47.59  smallcut_100k pp    3.57  batch_256 pp   18.86
//   Dijkstra_SK 256 to 2000 512 to 5000 work 400000: pareto_100k pp   45.59  smallcut_100k pp    3.59  batch_256 pp   18.87
//   Dijkstra_SK 256 to 2000 512 to 5000 work 200000: pareto_100k pp   45.52  smallcut_100k pp    3.64  batch_256 pp   18.91
//   Dijkstra_SK 256 to 2000 512 to 5000 work 100000: pareto_100k pp   45.71  smallcut_100k pp    3.59  batch_256 pp   18.86
//   Dijkstra_SK 256 to 1000 512 to 2000 work      0: pareto_100k pp   45.98  smallcut_100k pp    3.59  batch_256 pp   18.89
//   Dijkstra_SK 256 to 1000 512 to 2000 work 400000: pareto_100k pp   45.45  smallcut_100k pp    3.55  batch_256 pp   18.88
//   Dijkstra_SK 256 to 1000 512 to 2000 work 200000: pareto_100k pp   45.45  smallcut_100k pp    3.61  batch_256 pp   18.90
//   Dijkstra_SK 256 to 1000 512 to 2000 work 100000: pareto_100k pp   45.84  smallcut_100k pp    3.72  batch_256 pp   19.12
//   Dijkstra_SK 256 to  500 512 to 1000 work      0: pareto_100k pp   45.57  smallcut_100k pp    3.68  batch_256 pp   19.00
//   Dijkstra_SK 256 to  500 512 to 1000 work 400000: pareto_100k pp   45.84  smallcut_100k pp    3.71  batch_256 pp   18.96
//   Dijkstra_SK 256 to  500 512 to 1000 work 200000: pareto_100k pp   45.70  smallcut_100k pp    3.72  batch_256 pp   19.09
//   Dijkstra_SK 256 to  500 512 to 1000 work 100000: pareto_100k pp   46.03  smallcut_100k pp    3.72  batch_256 pp   19.31
//   Dijkstra_SK 256 to  250 512 to 1000 work      0: pareto_100k pp   46.68  smallcut_100k pp    3.67  batch_256 pp   19.78
//   Dijkstra_SK 256 to  250 512 to 1000 work 400000: pareto_100k pp   46.05  smallcut_100k pp    3.57  batch_256 pp   19.71
//   Dijkstra_SK 256 to  250 512 to 1000 work 200000: pareto_100k pp   45.98  smallcut_100k pp    3.61  batch_256 pp   19.57
//   Dijkstra_SK 256 to  250 512 to 1000 work 100000: pareto_100k pp   46.39  smallcut_100k pp    3.59  batch_256 pp   19.72
//   Dijkstra_SK 256 to  500 512 to 2000 work      0: pareto_100k pp   45.95  smallcut_100k pp    3.61  batch_256 pp   18.96
//   Dijkstra_SK 256 to  500 512 to 2000 work 400000: pareto_100k pp   45.51  smallcut_100k pp    3.61  batch_256 pp   18.99
//   Dijkstra_SK 256 to  500 512 to 2000 work 200000: pareto_100k pp   46.12  smallcut_100k pp    3.61  batch_256 pp   18.91
//   Dijkstra_SK 256 to  500 512 to 2000 work 100000: pareto_100k pp   45.85  smallcut_100k pp    3.59  batch_256 pp   19.27
//   chosen: small range 2000, mid range 6000, sources-per-group divisor 256, dense shift 1, Dijkstra_SK small 1000 mid 2000 work 400000
#pragma once
#include <cstdint>

namespace bcpp {
constexpr int64_t tuned_small_range = 2000;
constexpr int64_t tuned_mid_range = 6000;
constexpr int64_t tuned_spg_div = 256;
constexpr int64_t tuned_dense_shift = 1;
constexpr int64_t tuned_dsk_small_range = 1000;
constexpr int64_t tuned_dsk_mid_range = 2000;
constexpr int64_t tuned_dsk_group_work = 400000;
}  // namespace bcpp
