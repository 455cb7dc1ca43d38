// Reverse sweep instantiations: FP32.
#include "rts_reverse.hpp"

namespace rts {
RTS_REV_INST(float)
}  // namespace rts
