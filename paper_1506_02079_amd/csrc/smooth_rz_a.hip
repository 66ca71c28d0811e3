// Smoothing kernel instances for cross-slice radii 0, 1, 2, 3, 4, 5 (see smooth_impl.h).
#include "smooth_impl.h"

namespace gdf {

GDF_SMOOTH_RZ(0)
GDF_SMOOTH_RZ(1)
GDF_SMOOTH_RZ(2)
GDF_SMOOTH_RZ(3)
GDF_SMOOTH_RZ(4)
GDF_SMOOTH_RZ(5)

}  // namespace gdf
