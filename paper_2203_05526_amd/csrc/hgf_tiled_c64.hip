// Instantiations of the tiled RK4 stage kernels and the resident integrator for float2 stage grids and a double2 state.
#include "hgf_resident.h"
#include "hgf_tiled.h"

namespace hgf {
HGF_TILED_INSTANTIATE(float2, double2, c64)
HGF_RESIDENT_INSTANTIATE(float2, double2, c64)
}  // namespace hgf
