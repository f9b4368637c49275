// History-based baseline: the event programs of runs without time bins.  Those
// of runs with time-binned tallies are built in sched_naive_time.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_naive.hpp"

namespace mcx {

hipError_t launch_naive(const LaunchArgs &a, LaunchStats &st, LaunchTimer &tm)
{
    return a.time ? launch_naive_time(a, st, tm) : launch_naive_tm<0>(a, st, tm);
}

}  // namespace mcx
