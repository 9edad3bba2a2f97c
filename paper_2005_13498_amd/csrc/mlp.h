// Launchers of the controller MLP kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hub {

int mlp_grad_waves(int n_rows);          // wavefronts (gradient partial rows) of one train step
int64_t mlp_workspace_bytes(int n_rows);  // device bytes of those partials
hipError_t launch_mlp_forward(const float* params, int n_rows, const float* feats, float* out, hipStream_t s);
hipError_t launch_mlp_train_step(float* params, float* m, float* v, int t, float lr, int n_rows, const float* feats,
                                 const float* targets, float* loss, void* workspace, hipStream_t s);

}  // namespace hub
