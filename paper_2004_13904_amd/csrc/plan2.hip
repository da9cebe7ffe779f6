// The operator's pass launchers with stage plan 2 of the FFTs (see plan_passes.h).
#define FF_PLAN_UNIT
#include "plan_passes.h"

namespace ff {
FF_PLAN_INSTANTIATE(2)
}  // namespace ff
