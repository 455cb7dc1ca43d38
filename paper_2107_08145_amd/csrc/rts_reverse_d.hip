// Reverse sweep instantiations: FP64.
#include "rts_reverse.hpp"

namespace rts {
RTS_REV_INST(double)
}  // namespace rts
