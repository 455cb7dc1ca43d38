// Forward sweep instantiations: FP32, 2 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(float, 2)
}  // namespace rts
