// Forward sweep instantiations: FP32, 6 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(float, 6)
}  // namespace rts
