// Internal launcher interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace prk {

hipError_t launch_plain(const Params& P, bool rec, hipStream_t st);
hipError_t launch_mixed(const Params& P, bool rec, int grid, int block, hipStream_t st);
int mixed_occupancy(const Params& P, int block);
int mixed_lds_bytes(const Params& P);
int mixed_max_block(const Params& P);   // the launch bound of the persistent kernel P selects
int batch_max_block(bool grid_nav);
hipError_t launch_batch(const BatchParams& B, bool slds, bool grid_nav, int grid, int block, hipStream_t st);
int batch_occupancy(const BatchParams& B, bool slds, bool grid_nav, int block);
int batch_lds_bytes(const BatchParams& B);
int batch_scene_lds_bytes(int nv, int nm, int nf, int nc, int ng, int ncs, int nci, int grid);
hipError_t zero_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t prepared_tail(unsigned long long* const* hist, const unsigned long long* add, int n,
                         unsigned long long* shift, unsigned long long stride, hipStream_t st);
hipError_t zero_f64(double* p, uint64_t n, hipStream_t st);

}  // namespace prk
