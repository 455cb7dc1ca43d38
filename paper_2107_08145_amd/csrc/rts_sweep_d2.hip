// Forward sweep instantiations: FP64, 2 rows per strip.
#include "rts_sweep.hpp"

namespace rts {
RTS_INST(double, 2)
}  // namespace rts
