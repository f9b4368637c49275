// Stack-based remapping: the event programs of runs with time bins or non-analog
// weights (extended particle state).
#include "sched_stack.hpp"

namespace mcx {

hipError_t launch_stack_ext(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return launch_stack_tm<1>(a, ws, st, tm, flag);
}

}  // namespace mcx
