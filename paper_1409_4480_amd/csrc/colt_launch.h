// Host-side launchers of the transport kernels (defined in colt_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "colt_internal.h"

namespace colt {

// rf_stride: CellRec<float> slots per cell (2 for octrees: links in the second half)
hipError_t launch_cell_setup(int64_t n, const double *n_HI, const double *T, const double *v,
                             const double *k_dust, const double *atau_nl, double dx_cm,
                             void *rd, void *ad, void *rf, int rf_stride, void *af, hipStream_t s);
// J1: the job of a one-job launch (L.n_jobs == 1), passed to the kernel by value
hipError_t launch_transport(int precision, bool cams, const LaunchView &L, const JobView &J1,
                            int grid, int block, hipStream_t s);
// grid_kind: the grid kind of a one-job launch (0 Cartesian, 1 octree)
hipError_t transport_occupancy(int precision, bool cams, bool single, int grid_kind, int block,
                               int *blocks_per_cu);
// k_plan (advance = false) before a transport launch, k_advance after it
hipError_t launch_plan(const LaunchView &L, bool advance, hipStream_t s);
hipError_t launch_peel(int precision, const JobView &J, unsigned long long *work, int grid,
                       hipStream_t s);
hipError_t peel_occupancy(int precision, int grid_kind, int *blocks_per_cu);
// The current device's fixed launch table for colt_transport_static (its
// address found once per device) and the kernel that writes job views into it.
hipError_t static_table(void **ptr);
hipError_t put_views(const JobView *views, int n, JobView *dst, hipStream_t s);
hipError_t launch_nonlocal(const GridView &g, const double *n_HI, const double *leaf_boxes,
                           int64_t n, double f_nl, void *ad, void *af, hipStream_t s);
hipError_t launch_voigt(int precision, int64_t n, const double *a, const double *x, double *out,
                        hipStream_t s);
hipError_t launch_sample(int precision, int what, double p0, double p1, double p2,
                         uint64_t seed, int64_t n, double *out, int32_t *draws, hipStream_t s);

}  // namespace colt
