// Asynchronous remapping: the event programs of runs without time bins.  Those
// of runs with time-binned tallies are built in sched_async_time.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_async.hpp"

namespace mcx {

hipError_t launch_async(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return a.time ? launch_async_time(a, ws, st, tm) : launch_async_tm<0>(a, ws, st, tm);
}

}  // namespace mcx
