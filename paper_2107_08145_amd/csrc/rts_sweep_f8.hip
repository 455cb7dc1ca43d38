// Forward sweep instantiations: FP32, 8 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(float, 8)
}  // namespace rts
