// Stack-based remapping: the event programs of runs with time-binned tallies.
#include "sched_stack.hpp"

namespace mcx {

hipError_t launch_stack_time(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return launch_stack_tm<1>(a, ws, st, tm, flag);
}

}  // namespace mcx
