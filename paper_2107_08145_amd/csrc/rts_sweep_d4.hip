// Forward sweep instantiations: FP64, 4 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(double, 4)
}  // namespace rts
