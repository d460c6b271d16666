// Single-problem path instantiated for one key codec (DT_I32).
#include "runner.h"

namespace drtopk {
template void run_codec<DT_I32>(const Plan&, const uint32_t*, void*, uint32_t*, uint32_t*, uint32_t*, bool, bool,
                                hipStream_t);
template void delegates_codec<DT_I32>(const Plan&, const uint32_t*, uint32_t*, uint32_t*, Ctl*, hipStream_t);
}  // namespace drtopk
