// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from
// timings on one MI355X; edit by re-running it, not by hand.
//
// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to
// tuned_mid_range with 512, larger ones with 1024. A group holds
// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes
// with more than n >> tuned_dense_shift bits scans the range instead.
//
// Timings of the sweep (ms, best of 2 after a warm-up run):
//   256 to 1500 512 to 4000 div  256: sbm_10k plain   10.56  sbm_10k pp   11.10  planted_1k plain    0.49  planted_1k pp    0.87  batch_256 plain    8.61  batch_256 pp   23.34
//   256 to 2000 512 to 5000 div  256: sbm_10k plain   10.43  sbm_10k pp   11.10  planted_1k plain    0.49  planted_1k pp    0.87  batch_256 plain    7.78  batch_256 pp   22.76
//   256 to 2000 512 to 6000 div  256: sbm_10k plain   10.50  sbm_10k pp   11.08  planted_1k plain    0.50  planted_1k pp    0.87  batch_256 plain    7.70  batch_256 pp   22.86
//   256 to 2500 512 to 5000 div  256: sbm_10k plain   10.46  sbm_10k pp   11.06  planted_1k plain    0.53  planted_1k pp    1.06  batch_256 plain    7.88  batch_256 pp   23.31
//   256 to 1500 512 to 5000 div  256: sbm_10k plain   10.45  sbm_10k pp   11.05  planted_1k plain    0.50  planted_1k pp    0.88  batch_256 plain    7.97  batch_256 pp   22.91
//   256 to 2000 512 to 4000 div  256: sbm_10k plain   10.43  sbm_10k pp   11.05  planted_1k plain    0.50  planted_1k pp    0.87  batch_256 plain    8.46  batch_256 pp   23.07
//   chosen: small range 2000, mid range 5000, sources-per-group divisor 256, dense shift 1
#pragma once
#include <cstdint>

namespace bcpp {
constexpr int64_t tuned_small_range = 2000;
constexpr int64_t tuned_mid_range = 5000;
constexpr int64_t tuned_spg_div = 256;
constexpr int64_t tuned_dense_shift = 1;
}  // namespace bcpp
