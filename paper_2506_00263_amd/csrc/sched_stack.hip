// Stack-based remapping: the event programs of runs without time bins.  Those
// of runs with time-binned tallies are built in sched_stack_time.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_stack.hpp"

namespace mcx {

hipError_t launch_stack(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return a.time ? launch_stack_time(a, ws, st, tm, flag) : launch_stack_tm<0>(a, ws, st, tm, flag);
}

}  // namespace mcx
