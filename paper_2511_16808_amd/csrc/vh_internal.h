// vh_internal.h -- interfaces between the library's translation units that are not part of
// the C ABI (include/vh.h).
#pragma once

#include <cstddef>

#include "../../include/vh.h"

// vh_setup building the handle inside a device region the caller owns: every device array
// of the handle (hierarchy, FGMRES and multi-source workspaces) is carved out of
// [region, region + region_bytes) without hipMalloc or hipFree, and vh_destroy returns
// nothing to the device allocator.  pinned: host-pinned status buffer of 4 + 256 doubles,
// owned by the caller, used by one handle at a time.  region_bytes must be at least
// vh_region_bytes() of the same arguments.
vh_status vh_setup_region(vh_handle** out, int dim, const int* n, double h, double omega,
                          const double* kappa, const double* gamma, double shift, int levels,
                          int patch, const vh_options* opt, void* region, size_t region_bytes,
                          double* pinned);

// Bytes of a region that holds the handle of vh_setup_region at its peak over set-up and
// a vh_solve of nsrc sources: vh_footprint_bytes plus the 256-byte alignment of every
// array carved out of the region.
size_t vh_region_bytes(int dim, const int* n, int levels, int patch, int nsrc,
                       const vh_options* opt);
