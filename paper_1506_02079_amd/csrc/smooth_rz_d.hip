// Smoothing kernel instances for cross-slice radii 10, 11, 12 (see smooth_impl.h).
#include "smooth_impl.h"

namespace gdf {

GDF_SMOOTH_RZ(10)
GDF_SMOOTH_RZ(11)
GDF_SMOOTH_RZ(12)

}  // namespace gdf
