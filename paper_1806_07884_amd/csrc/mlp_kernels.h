// Launch wrappers of the learned-radius kernels (features, MLP, broadcast).
#pragma once

#include "internal.h"

namespace rbf {

struct PlanView;

constexpr int kMlpInputs = 16;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpInputs * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;  // 5313
constexpr int kMaxRadii = 8;

hipError_t launch_density_counts(const PlanView& P, const double* radii, int R, int reach,
                                 int32_t* counts, hipStream_t s);
// box = {min_0, max_0, min_1, max_1, ...} of the centres (device)
hipError_t launch_centre_blocks(const double* ctr, int64_t m, int dim, const double* box, int nb,
                                int32_t* blk, hipStream_t s);
hipError_t launch_block_features(const int32_t* counts, const int32_t* blk, int64_t m, int R,
                                 int nblocks, float* feats, hipStream_t s);
hipError_t launch_block_sq_err(const double* y, int64_t nq, int dim, const double* f,
                               const double* h, const double* box, int nb, int nblocks,
                               double* sums, int64_t* counts, hipStream_t s);
hipError_t launch_radius_broadcast(const float* pred, const int32_t* blk, int64_t m,
                                   double spacing, double rho_min, double rho_max,
                                   double rho_fallback, double* rho, hipStream_t s);
// scale: device {mean[16], std[16]}; every input is standardised as
// (x_i - mean_i) / std_i in float32 when loaded.
hipError_t launch_mlp_grad(const float* params, const float* scale, const float* x,
                           const float* y, int64_t n, float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_train(float* params, float* m1, float* m2, const float* scale,
                            const float* x, const float* y, const int32_t* order, int steps,
                            int batch, float lr, int t0, float* losses, hipStream_t s);
hipError_t launch_mlp_infer_bf16(const float* params, const float* scale, const float* x,
                                 int64_t n, float* out, hipStream_t s);

}  // namespace rbf
