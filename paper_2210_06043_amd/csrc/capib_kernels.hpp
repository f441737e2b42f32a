// Host-side launchers of the libcapib kernels (internal).
#pragma once
#include <hip/hip_ext.h>

#include "capib_dev.hpp"

namespace capib {

// The step kernels take an optional pair of events that, when given, are
// stamped at the start and the end of the kernel's execution
// (hipExtLaunchKernelGGL), so that the elapsed time is the kernel alone.
hipError_t launch_lattice_far(const Dev &d, int par, hipStream_t st, hipEvent_t e0 = nullptr,
                              hipEvent_t e1 = nullptr);
// pct: percent of each XCD's run of far-tile candidates that the membrane
// launch swept (the sweep takes the rest)
hipError_t launch_lattice_sweep(const Dev &d, int par, hipStream_t st, hipEvent_t e0 = nullptr,
                                hipEvent_t e1 = nullptr, int pct = 0);
// whether the far tiles are swept beside the membrane phase (Dev::split)
bool lattice_split(const Dev &d);
// the library's own rules for the launch configuration: the far tiles beside
// the membrane phase on lattices of 8192 tiles or more; the marking with
// (vertex, tile) pairs below 16384 vertices; the membrane launch's far share
bool default_split(int tiles);
bool default_mark_pairs(int nverts);
int default_far_share(int storage);
hipError_t launch_mark(const Dev &d, int par, hipStream_t st);
hipError_t launch_macro(const Dev &d, int par, hipStream_t st);
hipError_t launch_init_flow(const Dev &d, int par, hipStream_t st);
hipError_t launch_diag(const Dev &d, int par, hipStream_t st);

hipError_t launch_interp(const Dev &d, int par, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_body(const Dev &d, int par, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// On a lattice below SPLIT_MIN_TILES tiles: the membrane kernel with the
// first body_far_share(d) percent of each XCD's run of far-tile candidates
// in the same launch, then the sweep takes the rest (launch_lattice_sweep
// with that percentage).
int body_far_share(const Dev &d);
hipError_t launch_body_far(const Dev &d, int par, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_census(const Dev &d, int par, int pct, unsigned long long *out, hipStream_t st);
hipError_t launch_body_geom(const Dev &d, int par, hipStream_t st);
hipError_t launch_sample(const Dev &d, int par, int ptag, int ctag, float *out, hipStream_t st);

}  // namespace capib
