// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from
// timings on one MI355X; edit by re-running it, not by hand.
//
// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to
// tuned_mid_range with 512, larger ones with 1024. A group holds
// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes
// with more than n >> tuned_dense_shift bits scans the range instead.
//
// Timings of the sweep (ms, best of 2 after a warm-up run):
//   256 to  all 512 to  all div  256: sbm_10k plain   36.37  sbm_10k pp   36.99  planted_1k plain    0.62  planted_1k pp    0.97  batch_256 plain   19.25  batch_256 pp   57.06
//   256 to  all 512 to  all div 1024: sbm_10k plain   36.76  sbm_10k pp   37.27  planted_1k plain    0.79  planted_1k pp    1.15  batch_256 plain   19.69  batch_256 pp   58.97
//   256 to  all 512 to  all div 4096: sbm_10k plain   40.38  sbm_10k pp   41.00  planted_1k plain    0.79  planted_1k pp    1.16  batch_256 plain   19.67  batch_256 pp   58.51
//   256 to 6500 512 to  all div  256: sbm_10k plain   22.46  sbm_10k pp   22.99  planted_1k plain    0.60  planted_1k pp    1.00  batch_256 plain   19.18  batch_256 pp   57.27
//   256 to 6500 512 to  all div 1024: sbm_10k plain   22.70  sbm_10k pp   23.23  planted_1k plain    0.78  planted_1k pp    1.10  batch_256 plain   19.64  batch_256 pp   58.46
//   256 to 6500 512 to  all div 4096: sbm_10k plain   25.99  sbm_10k pp   26.41  planted_1k plain    0.77  planted_1k pp    1.09  batch_256 plain   19.69  batch_256 pp   58.62
//   256 to 4000 512 to 6500 div  256: sbm_10k plain   16.08  sbm_10k pp   16.61  planted_1k plain    0.59  planted_1k pp    0.93  batch_256 plain   13.24  batch_256 pp   46.67
//   256 to 4000 512 to 6500 div 1024: sbm_10k plain   16.24  sbm_10k pp   16.87  planted_1k plain    0.77  planted_1k pp    1.10  batch_256 plain   13.74  batch_256 pp   47.56
//   256 to 4000 512 to 6500 div 4096: sbm_10k plain   19.14  sbm_10k pp   19.79  planted_1k plain    0.77  planted_1k pp    1.11  batch_256 plain   13.77  batch_256 pp   47.32
//   256 to 2500 512 to 6500 div  256: sbm_10k plain   16.07  sbm_10k pp   16.71  planted_1k plain    0.59  planted_1k pp    0.94  batch_256 plain   11.65  batch_256 pp   41.74
//   256 to 2500 512 to 6500 div 1024: sbm_10k plain   16.23  sbm_10k pp   16.81  planted_1k plain    0.78  planted_1k pp    1.09  batch_256 plain   12.05  batch_256 pp   43.08
//   256 to 2500 512 to 6500 div 4096: sbm_10k plain   19.20  sbm_10k pp   19.72  planted_1k plain    0.78  planted_1k pp    1.09  batch_256 plain   12.03  batch_256 pp   42.91
//   256 to 2500 512 to 2500 div  256: sbm_10k plain   16.09  sbm_10k pp   16.64  planted_1k plain    0.58  planted_1k pp    0.93  batch_256 plain   13.95  batch_256 pp   45.19
//   256 to 2500 512 to 2500 div 1024: sbm_10k plain   16.24  sbm_10k pp   16.84  planted_1k plain    0.77  planted_1k pp    1.11  batch_256 plain   14.46  batch_256 pp   47.52
//   256 to 2500 512 to 2500 div 4096: sbm_10k plain   19.19  sbm_10k pp   19.74  planted_1k plain    0.77  planted_1k pp    1.08  batch_256 plain   14.48  batch_256 pp   47.42
//   256 to 1000 512 to 4000 div  256: sbm_10k plain   16.11  sbm_10k pp   16.68  planted_1k plain    0.59  planted_1k pp    0.92  batch_256 plain   13.82  batch_256 pp   44.62
//   256 to 1000 512 to 4000 div 1024: sbm_10k plain   16.22  sbm_10k pp   16.82  planted_1k plain    0.77  planted_1k pp    1.08  batch_256 plain   14.51  batch_256 pp   46.04
//   256 to 1000 512 to 4000 div 4096: sbm_10k plain   19.18  sbm_10k pp   19.74  planted_1k plain    0.76  planted_1k pp    1.05  batch_256 plain   14.49  batch_256 pp   45.92
//   256 to    0 512 to 6500 div  256: sbm_10k plain   16.12  sbm_10k pp   16.70  planted_1k plain    0.59  planted_1k pp    0.93  batch_256 plain   13.24  batch_256 pp   46.92
//   256 to    0 512 to 6500 div 1024: sbm_10k plain   16.31  sbm_10k pp   16.88  planted_1k plain    0.79  planted_1k pp    1.12  batch_256 plain   13.73  batch_256 pp   47.30
//   256 to    0 512 to 6500 div 4096: sbm_10k plain   19.16  sbm_10k pp   19.76  planted_1k plain    0.77  planted_1k pp    1.12  batch_256 plain   13.75  batch_256 pp   47.77
//   256 to    0 512 to 2500 div  256: sbm_10k plain   16.05  sbm_10k pp   16.77  planted_1k plain    0.59  planted_1k pp    0.94  batch_256 plain   14.19  batch_256 pp   47.32
//   256 to    0 512 to 2500 div 1024: sbm_10k plain   16.29  sbm_10k pp   16.84  planted_1k plain    0.78  planted_1k pp    1.11  batch_256 plain   14.90  batch_256 pp   48.19
//   256 to    0 512 to 2500 div 4096: sbm_10k plain   19.22  sbm_10k pp   19.77  planted_1k plain    0.79  planted_1k pp    1.10  batch_256 plain   14.92  batch_256 pp   48.09
//   256 to    0 512 to    0 div  256: sbm_10k plain   16.07  sbm_10k pp   16.66  planted_1k plain    0.58  planted_1k pp    0.93  batch_256 plain   13.21  batch_256 pp   46.80
//   256 to    0 512 to    0 div 1024: sbm_10k plain   16.26  sbm_10k pp   16.86  planted_1k plain    0.77  planted_1k pp    1.08  batch_256 plain   13.76  batch_256 pp   47.53
//   256 to    0 512 to    0 div 4096: sbm_10k plain   19.15  sbm_10k pp   19.72  planted_1k plain    0.77  planted_1k pp    1.10  batch_256 plain   13.76  batch_256 pp   47.54
//   dense shift  1: smallcut_100k plain    6.443 ms  smallcut_100k pp    3.884 ms  pareto_100k plain   50.290 ms  pareto_100k pp  108.664 ms
//   dense shift  2: smallcut_100k plain    6.424 ms  smallcut_100k pp    3.648 ms  pareto_100k plain   50.728 ms  pareto_100k pp  109.910 ms
//   dense shift  3: smallcut_100k plain    6.392 ms  smallcut_100k pp    3.640 ms  pareto_100k plain   50.990 ms  pareto_100k pp  110.989 ms
//   dense shift  4: smallcut_100k plain    6.646 ms  smallcut_100k pp    3.749 ms  pareto_100k plain   51.498 ms  pareto_100k pp  109.792 ms
//   dense shift  6: smallcut_100k plain    6.972 ms  smallcut_100k pp    3.713 ms  pareto_100k plain   51.881 ms  pareto_100k pp  110.050 ms
//   dense shift 63: smallcut_100k plain    8.700 ms  smallcut_100k pp    3.693 ms  pareto_100k plain   54.129 ms  pareto_100k pp  112.353 ms
//   chosen: small range 2500, mid range 6500, sources-per-group divisor 256, dense shift 2
#pragma once
#include <cstdint>

namespace bcpp {
constexpr int64_t tuned_small_range = 2500;
constexpr int64_t tuned_mid_range = 6500;
constexpr int64_t tuned_spg_div = 256;
constexpr int64_t tuned_dense_shift = 2;
}  // namespace bcpp
