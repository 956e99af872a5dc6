// Instantiations of the tiled RK4 stage kernels and the resident integrator for double stage grids and a double state.
#include "hgf_resident.h"
#include "hgf_tiled.h"

namespace hgf {
HGF_TILED_INSTANTIATE(double, double, r64)
HGF_RESIDENT_INSTANTIATE(double, double, r64)
}  // namespace hgf
