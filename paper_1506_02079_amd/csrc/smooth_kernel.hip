// Dispatch of the anisotropic smoothing kernel over its compile-time radii.
#include "internal.h"

namespace gdf {

#define GDF_DECL(RZ) hipError_t smooth_rz_##RZ(bool fp64, const SmoothArgs &a, hipStream_t s);
GDF_DECL(0) GDF_DECL(1) GDF_DECL(2) GDF_DECL(3) GDF_DECL(4) GDF_DECL(5) GDF_DECL(6)
GDF_DECL(7) GDF_DECL(8) GDF_DECL(9) GDF_DECL(10) GDF_DECL(11) GDF_DECL(12)
#undef GDF_DECL

hipError_t launch_smooth(bool fp64, const SmoothArgs &a, hipStream_t s)
{
    if (a.rxy > 7 || a.rz > 12 || a.rxy < 0 || a.rz < 0) return hipErrorInvalidValue;
    switch (a.rz) {
#define GDF_CASE(RZ) case RZ: return smooth_rz_##RZ(fp64, a, s);
        GDF_CASE(0) GDF_CASE(1) GDF_CASE(2) GDF_CASE(3) GDF_CASE(4) GDF_CASE(5) GDF_CASE(6)
        GDF_CASE(7) GDF_CASE(8) GDF_CASE(9) GDF_CASE(10) GDF_CASE(11) GDF_CASE(12)
#undef GDF_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace gdf
