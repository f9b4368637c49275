// Asynchronous remapping: the event programs of runs with time-binned tallies.
#include "sched_async.hpp"

namespace mcx {

hipError_t launch_async_time(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm)
{
    return launch_async_tm<1>(a, ws, st, tm);
}

}  // namespace mcx
