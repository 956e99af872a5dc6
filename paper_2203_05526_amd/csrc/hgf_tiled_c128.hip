// Instantiations of the tiled RK4 stage kernels and the resident integrator for double2 stage grids and a double2 state.
#include "hgf_resident.h"
#include "hgf_tiled.h"

namespace hgf {
HGF_TILED_INSTANTIATE(double2, double2, c128)
HGF_RESIDENT_INSTANTIATE(double2, double2, c128)
HGF_ADJOINT_RESIDENT_DEFINE()
}  // namespace hgf
