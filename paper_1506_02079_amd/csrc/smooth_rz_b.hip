// Smoothing kernel instances for cross-slice radii 6, 7, 8 (see smooth_impl.h).
#include "smooth_impl.h"

namespace gdf {

GDF_SMOOTH_RZ(6)
GDF_SMOOTH_RZ(7)
GDF_SMOOTH_RZ(8)

}  // namespace gdf
