// History-based baseline: the event programs of runs whose particles carry no
// extended state.  Those of runs with time bins or non-analog weights
// (particle time and weight in the bank) are built in sched_naive_ext.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_naive.hpp"

namespace mcx {

hipError_t launch_naive(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    return a.ext ? launch_naive_ext(a, st, tm) : launch_naive_tm<0>(a, st, tm);
}

}  // namespace mcx
