// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from
// timings on one MI355X; edit by re-running it, not by hand.
//
// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to
// tuned_mid_range with 512, larger ones with 1024. A group holds
// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes
// with more than n >> tuned_dense_shift bits scans the range instead.
//
// Timings of the sweep (ms, best of 2 after a warm-up run):
//   256 to  all 512 to  all div  256: sbm_10k plain   29.69  sbm_10k pp   30.24  planted_1k plain    0.49  planted_1k pp    0.87  batch_256 plain   14.34  batch_256 pp   38.61
//   256 to  all 512 to  all div 1024: sbm_10k plain   29.91  sbm_10k pp   30.53  planted_1k plain    0.77  planted_1k pp    1.14  batch_256 plain   14.98  batch_256 pp   37.87
//   256 to 6500 512 to  all div  256: sbm_10k plain   17.78  sbm_10k pp   18.35  planted_1k plain    0.49  planted_1k pp    0.88  batch_256 plain   14.26  batch_256 pp   38.57
//   256 to 6500 512 to  all div 1024: sbm_10k plain   18.09  sbm_10k pp   18.66  planted_1k plain    0.75  planted_1k pp    1.11  batch_256 plain   14.83  batch_256 pp   37.87
//   256 to 4000 512 to 6500 div  256: sbm_10k plain   12.64  sbm_10k pp   13.16  planted_1k plain    0.48  planted_1k pp    0.87  batch_256 plain   10.02  batch_256 pp   30.62
//   256 to 4000 512 to 6500 div 1024: sbm_10k plain   13.03  sbm_10k pp   13.56  planted_1k plain    0.75  planted_1k pp    1.02  batch_256 plain   10.48  batch_256 pp   29.02
//   256 to 2500 512 to 6500 div  256: sbm_10k plain   12.65  sbm_10k pp   13.25  planted_1k plain    0.49  planted_1k pp    0.88  batch_256 plain    8.74  batch_256 pp   26.52
//   256 to 2500 512 to 6500 div 1024: sbm_10k plain   13.02  sbm_10k pp   13.58  planted_1k plain    0.75  planted_1k pp    1.02  batch_256 plain    9.25  batch_256 pp   25.44
//   256 to 2500 512 to 4000 div  256: sbm_10k plain   12.66  sbm_10k pp   13.22  planted_1k plain    0.49  planted_1k pp    0.88  batch_256 plain    9.03  batch_256 pp   24.87
//   256 to 2500 512 to 4000 div 1024: sbm_10k plain   13.01  sbm_10k pp   13.58  planted_1k plain    0.75  planted_1k pp    1.11  batch_256 plain    9.43  batch_256 pp   23.91
//   256 to 1500 512 to 6500 div  256: sbm_10k plain   12.64  sbm_10k pp   13.28  planted_1k plain    0.49  planted_1k pp    0.88  batch_256 plain    9.09  batch_256 pp   26.77
//   256 to 1500 512 to 6500 div 1024: sbm_10k plain   13.04  sbm_10k pp   13.61  planted_1k plain    0.75  planted_1k pp    1.11  batch_256 plain    9.59  batch_256 pp   26.11
//   256 to 1500 512 to 4000 div  256: sbm_10k plain   12.64  sbm_10k pp   13.20  planted_1k plain    0.49  planted_1k pp    0.88  batch_256 plain    8.80  batch_256 pp   24.25
//   256 to 1500 512 to 4000 div 1024: sbm_10k plain   13.03  sbm_10k pp   13.60  planted_1k plain    0.74  planted_1k pp    1.12  batch_256 plain    9.43  batch_256 pp   23.37
//   256 to 1000 512 to 6500 div  256: sbm_10k plain   12.65  sbm_10k pp   13.24  planted_1k plain    0.49  planted_1k pp    0.87  batch_256 plain    9.34  batch_256 pp   27.28
//   256 to 1000 512 to 6500 div 1024: sbm_10k plain   13.05  sbm_10k pp   13.58  planted_1k plain    0.76  planted_1k pp    1.09  batch_256 plain    9.95  batch_256 pp   26.72
//   256 to 1000 512 to 4000 div  256: sbm_10k plain   12.64  sbm_10k pp   13.23  planted_1k plain    0.48  planted_1k pp    0.90  batch_256 plain    8.89  batch_256 pp   24.31
//   256 to 1000 512 to 4000 div 1024: sbm_10k plain   13.04  sbm_10k pp   13.63  planted_1k plain    0.74  planted_1k pp    1.10  batch_256 plain    9.47  batch_256 pp   23.40
//   256 to  500 512 to 4000 div  256: sbm_10k plain   12.62  sbm_10k pp   13.23  planted_1k plain    0.43  planted_1k pp    0.80  batch_256 plain    9.01  batch_256 pp   25.20
//   256 to  500 512 to 4000 div 1024: sbm_10k plain   13.04  sbm_10k pp   13.62  planted_1k plain    0.76  planted_1k pp    1.15  batch_256 plain    9.53  batch_256 pp   24.43
//   256 to    0 512 to 6500 div  256: sbm_10k plain   12.63  sbm_10k pp   13.25  planted_1k plain    0.43  planted_1k pp    0.81  batch_256 plain    9.70  batch_256 pp   28.86
//   256 to    0 512 to 6500 div 1024: sbm_10k plain   13.02  sbm_10k pp   13.64  planted_1k plain    0.76  planted_1k pp    1.02  batch_256 plain   10.22  batch_256 pp   28.42
//   256 to    0 512 to 4000 div  256: sbm_10k plain   12.60  sbm_10k pp   13.20  planted_1k plain    0.45  planted_1k pp    0.82  batch_256 plain    9.00  batch_256 pp   25.43
//   256 to    0 512 to 4000 div 1024: sbm_10k plain   13.02  sbm_10k pp   13.60  planted_1k plain    0.76  planted_1k pp    1.13  batch_256 plain    9.63  batch_256 pp   24.74
//   256 to    0 512 to    0 div  256: sbm_10k plain   12.63  sbm_10k pp   13.23  planted_1k plain    0.40  planted_1k pp    0.77  batch_256 plain   12.68  batch_256 pp   40.32
//   256 to    0 512 to    0 div 1024: sbm_10k plain   13.02  sbm_10k pp   13.63  planted_1k plain    0.83  planted_1k pp    1.22  batch_256 plain   13.32  batch_256 pp   40.58
//   dense shift  1: smallcut_100k plain    6.020 ms  smallcut_100k pp    3.363 ms  pareto_100k plain   48.917 ms  pareto_100k pp  103.363 ms
//   dense shift  2: smallcut_100k plain    5.985 ms  smallcut_100k pp    3.336 ms  pareto_100k plain   49.270 ms  pareto_100k pp  103.922 ms
//   dense shift  3: smallcut_100k plain    6.007 ms  smallcut_100k pp    3.378 ms  pareto_100k plain   49.627 ms  pareto_100k pp  104.081 ms
//   dense shift  4: smallcut_100k plain    6.250 ms  smallcut_100k pp    3.356 ms  pareto_100k plain   50.033 ms  pareto_100k pp  105.127 ms
//   dense shift  6: smallcut_100k plain    6.581 ms  smallcut_100k pp    3.361 ms  pareto_100k plain   50.503 ms  pareto_100k pp  105.305 ms
//   dense shift 63: smallcut_100k plain    8.387 ms  smallcut_100k pp    3.334 ms  pareto_100k plain   52.751 ms  pareto_100k pp  106.541 ms
//   chosen: small range 1500, mid range 4000, sources-per-group divisor 256, dense shift 1
#pragma once
#include <cstdint>

namespace bcpp {
constexpr int64_t tuned_small_range = 1500;
constexpr int64_t tuned_mid_range = 4000;
constexpr int64_t tuned_spg_div = 256;
constexpr int64_t tuned_dense_shift = 1;
}  // namespace bcpp
