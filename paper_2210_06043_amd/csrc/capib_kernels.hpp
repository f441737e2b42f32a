// Host-side launchers of the libcapib kernels (internal).
#pragma once
#include "capib_dev.hpp"

namespace capib {

hipError_t launch_lattice(const Dev &d, int par, hipStream_t st);
hipError_t launch_macro(const Dev &d, int par, hipStream_t st);
hipError_t launch_init_flow(const Dev &d, int par, hipStream_t st);
hipError_t launch_diag(const Dev &d, int par, hipStream_t st);

hipError_t launch_interp(const Dev &d, int par, hipStream_t st);
hipError_t launch_body(const Dev &d, int par, hipStream_t st);
hipError_t launch_body_geom(const Dev &d, int par, hipStream_t st);

}  // namespace capib
