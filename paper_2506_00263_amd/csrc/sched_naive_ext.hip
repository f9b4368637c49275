// History-based baseline: the event programs of runs with time bins or non-analog
// weights (extended particle state).
#include "sched_naive.hpp"

namespace mcx {

hipError_t launch_naive_ext(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    return launch_naive_tm<1>(a, st, tm);
}

}  // namespace mcx
