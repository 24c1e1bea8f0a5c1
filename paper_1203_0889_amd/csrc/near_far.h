// Internal interface of the mixed-precision near/far field stage: the device
// work queue that runs P2P (FP32 VALU) and M2L (FP32 MFMA) tasks.
#pragma once

#include "../../include/fmm.h"
#include "tree.h"

namespace fmm {

struct NearFarArgs {
    Geometry g;
    int32_t ncell;
    int64_t nleaf, n;
    int p;
    const int32_t *m2l_ptr, *m2l_src, *p2p_ptr, *p2p_src;
    const double *xs, *ys, *zs, *qs;
    const double *M;   // FP64 multipoles (input)
    double *L;         // FP64 locals (output, overwritten)
    double *phi, *fld; // FP64 near field per sorted particle (output)
    fmm_tuning tuning;
};

// Device workspaces owned by the plan for this stage.
struct NearFarState {
    DevBuf buf[16];
};

fmm_tuning default_tuning();
void run_near_far_mixed(NearFarState &st, const NearFarArgs &a, hipStream_t s);
void release_near_far(NearFarState &st);

}  // namespace fmm
