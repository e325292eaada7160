// Launch-shape defaults (overridden by the autotuner's cache when present).
#include "sv_internal.h"

namespace sv {

int default_max_local(sv_dtype dt) { return dt == SV_C128 ? 12 : 13; }

}  // namespace sv
