// Smoothing kernel instances for cross-slice radius 12 (see smooth_impl.h).
#include "smooth_impl.h"

namespace gdf {

GDF_SMOOTH_RZ(12)

}  // namespace gdf
