// Plan object behind ss_plan_t (internal to the library).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/sparstencil.h"
#include "kargs.hpp"

struct ss_plan_ {
    ss_plan_info info{};
    int ndim = 2;
    int64_t dims[3] = {1, 1, 1};      // slowest first; leading 1s for 1-D / 2-D
    int dtype = 0, boundary = 0, engine = 0, fuse = 1;
    int k = 3, rad = 1;               // of the (composed) stencil the kernels apply
    std::vector<double> w;            // (composed) coefficients, k^ndim
    // canonical tables
    std::vector<int32_t> perm;
    std::vector<double> values;
    std::vector<uint8_t> meta;
    std::vector<uint16_t> hi, lo, mid;   // mid: three-part states only
    std::vector<int32_t> lut;
    std::vector<double> model;        // rows of 7
    std::vector<int32_t> kernel_lut;
    std::vector<int32_t> kperm;       // A' column per K slot of the launched kernel
    std::vector<uint8_t> kernel_frags; // SS_Q_KERNEL_FRAGS: the kernel's A fragments
    // device
    void *dev = nullptr;
    ss::MmaArgs margs{};
    ss::MmaLaunch mma = nullptr;
    ss::DirectArgs dargs{};
    int device = 0;
    bool host_only = false;
    uint64_t klass = 0;               // equal for plans with identical device tables
    ss_plan_ *rem = nullptr;          // unfused plan for leftover sweeps
    // small 2-D FP64 grids on the direct engine: run() applies up to tb
    // sweeps per launch (temporal blocking); 0 = one sweep per launch
    int tb = 0;
    // two fused sweeps on a 2-D zero-halo grid: the band within edge_rad of
    // an edge is recomputed exactly from the unfused coefficients
    std::vector<double> w1;           // unfused coefficients
    int edge_rad = 0;
    double *edge_w = nullptr;         // device copy of w1 in FP64, then in FP32
    float *edge_w32 = nullptr;        // the FP32 copy (inside edge_w's allocation)
};

namespace ss {

// One sweep over n grids (n <= kMaxJobs) of plans of p's class: one launch.
hipError_t sweep_grids(const ss_plan_ *p, int n, const void *const *in, void *const *out,
                       const int64_t (*dims)[3], hipStream_t s);
hipError_t sweep_one(const ss_plan_ *p, const void *in, void *out, hipStream_t s);
bool band_in_launch(const ss_plan_ *p);
size_t plan_state_bytes(const ss_plan_ *p);
// True when a and b can share one launch: equal device tables and the same
// kernel (a plan of the direct engine picks its kernel from its grid size).
bool same_class(const ss_plan_ *a, const ss_plan_ *b);

}  // namespace ss
