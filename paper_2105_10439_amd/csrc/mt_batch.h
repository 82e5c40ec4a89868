// Internal interface of the batched multi-task fit (serve.hip) for the multi-task
// entry points (cofem.hip).  Not part of the public ABI.
//
// The L tasks (Sec. III-E.1) run as one alpha group of the serving kernels: every CG
// step of all L (K + 1) systems is one launch per phase, each task keeps its own
// dictionary, observation, probes (seed + l) and stop rule, and the joint M-step
// alpha_j = L / sum_l (mu_lj^2 + s_lj) runs on the device once all L E-steps of an
// EM iteration have ended.  Dense FP32 dictionaries, no refinement, K <= 31.
#pragma once
#include <hip/hip_runtime.h>

#include "cofem.h"

namespace cofem {

struct MtBatch;

// Whether the settings in p can run batched.
bool mtb_eligible(const cofem_params& p);
// Allocate the L task workspaces and capture the launch graph on `stream`.
cofem_status mtb_create(const cofem_params& p, int L, hipStream_t stream, MtBatch** out);
void mtb_destroy(MtBatch* b);
// Copy task `task`'s N x D row-major FP32 dictionary (device) into its workspace.
cofem_status mtb_set_dictionary(MtBatch* b, int task, const float* phi);
// The multi-task EM; ys holds L device pointers of N observations each.
cofem_status mtb_fit(MtBatch* b, const float* const* ys);
// Task `task`'s mu and s, the shared alpha (device buffers of D floats, any may be NULL)
// and its record.
cofem_status mtb_posterior(MtBatch* b, int task, float* mu, float* s, float* alpha, cofem_stats* st);

}  // namespace cofem
