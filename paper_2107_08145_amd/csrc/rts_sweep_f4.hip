// Forward sweep instantiations: FP32, 4 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(float, 4)
}  // namespace rts
