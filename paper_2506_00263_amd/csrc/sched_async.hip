// Asynchronous remapping: the event programs of runs whose particles carry no
// extended state.  Those of runs with time bins or non-analog weights
// (particle time and weight in the bank) are built in sched_async_ext.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_async.hpp"

namespace mcx {

hipError_t launch_async(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return a.ext ? launch_async_ext(a, ws, st, tm) : launch_async_tm<0>(a, ws, st, tm);
}

}  // namespace mcx
