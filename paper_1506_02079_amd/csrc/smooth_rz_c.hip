// Smoothing kernel instances for cross-slice radii 9 (see smooth_impl.h).
#include "smooth_impl.h"

namespace gdf {

GDF_SMOOTH_RZ(9)

}  // namespace gdf
