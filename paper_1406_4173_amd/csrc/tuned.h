// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from
// timings on one MI355X; edit by re-running it, not by hand.
//
// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to
// tuned_mid_range with 512, larger ones with 1024. A group holds
// ceil(|S| / tuned_spg_div) sources (1..64).
//
// Timings of the sweep (best of 3, plain target-set Brandes on the device):
//   n=   500 w=unit  T=256:    0.484 ms  T=512:    0.463 ms  T=1024:    0.511 ms
//   n=   500 w=1..10 T=256:    0.543 ms  T=512:    0.532 ms  T=1024:    0.622 ms
//   n=  1500 w=unit  T=256:    0.891 ms  T=512:    0.934 ms  T=1024:    1.045 ms
//   n=  1500 w=1..10 T=256:    0.972 ms  T=512:    1.035 ms  T=1024:    1.260 ms
//   n=  3000 w=unit  T=256:    1.011 ms  T=512:    1.070 ms  T=1024:    1.177 ms
//   n=  3000 w=1..10 T=256:    1.136 ms  T=512:    1.240 ms  T=1024:    1.434 ms
//   n=  5000 w=unit  T=256:    1.559 ms  T=512:    1.300 ms  T=1024:    1.409 ms
//   n=  5000 w=1..10 T=256:    1.866 ms  T=512:    1.522 ms  T=1024:    1.779 ms
//   n=  8000 w=unit  T=256:    3.181 ms  T=512:    2.211 ms  T=1024:    1.728 ms
//   n=  8000 w=1..10 T=256:    3.988 ms  T=512:    2.729 ms  T=1024:    2.131 ms
//   n= 12000 w=unit  T=256:    4.285 ms  T=512:    2.843 ms  T=1024:    2.101 ms
//   n= 12000 w=1..10 T=256:    5.520 ms  T=512:    3.572 ms  T=1024:    2.655 ms
//   best threads per size: 500: 512, 1500: 256, 3000: 256, 5000: 512, 8000: 1024, 12000: 1024
//   div=  256 sbm_10k plain   16.874 ms  batch_256 plain   16.202 ms
//   div=  512 sbm_10k plain   16.807 ms  batch_256 plain   17.828 ms
//   div= 1024 sbm_10k plain   16.931 ms  batch_256 plain   18.895 ms
//   div= 2048 sbm_10k plain   17.522 ms  batch_256 plain   18.715 ms
//   div= 4096 sbm_10k plain   18.899 ms  batch_256 plain   18.829 ms
//   chosen: small range 4000, mid range 6500, sources-per-group divisor 256
#pragma once
#include <cstdint>

namespace bcpp {
constexpr int64_t tuned_small_range = 4000;
constexpr int64_t tuned_mid_range = 6500;
constexpr int64_t tuned_spg_div = 256;
constexpr int64_t tuned_dense_shift = 2;
}  // namespace bcpp
