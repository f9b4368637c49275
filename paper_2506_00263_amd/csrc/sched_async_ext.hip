// Asynchronous remapping: the event programs of runs with time bins or non-analog
// weights (extended particle state).
#include "sched_async.hpp"

namespace mcx {

hipError_t launch_async_ext(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return launch_async_tm<1>(a, ws, st, tm);
}

}  // namespace mcx
