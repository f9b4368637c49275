// Stack-based remapping: the event programs of runs whose particles carry no
// extended state.  Those of runs with time bins or non-analog weights
// (particle time and weight in the bank) are built in sched_stack_ext.hip, a
// translation unit of their own that compiles in parallel.
#include "sched_stack.hpp"

namespace mcx {

hipError_t launch_stack(const LaunchArgs &a, Workspace &ws, LaunchStats &st, LaunchTimer &tm, unsigned int *flag)
{
    return a.ext ? launch_stack_ext(a, ws, st, tm, flag) : launch_stack_tm<0>(a, ws, st, tm, flag);
}

}  // namespace mcx
