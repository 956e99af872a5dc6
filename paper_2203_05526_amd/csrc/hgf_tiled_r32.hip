// Instantiations of the tiled RK4 stage kernels and the resident integrator for float stage grids and a double state.
#include "hgf_resident.h"
#include "hgf_tiled.h"

namespace hgf {
HGF_TILED_INSTANTIATE(float, double, r32)
HGF_RESIDENT_INSTANTIATE(float, double, r32)
}  // namespace hgf
