// Learned correction to the diagonal Davidson preconditioner.
//
// A per-element network maps 12 features of element i of the two-site
// vector to g_i and the correction is t_i = d_i r_i exp(clamp(g_i, -3, 3))
// with d_i = 1 / (theta - H_ii) (|theta - H_ii| clamped to >= 1e-12).
// Network: 12 -> 64 tanh -> 64 tanh -> 1; parameters in one FP32 vector
// ordered W1 (64 x 12, row-major), b1, W2 (64 x 64), b2, w3, b3.
// Features: 0 (theta - H_ii) / max(1, |theta|); 1 log(max(|theta - H_ii|,
// 1e-12)) / 10; 2 r_i sqrt(n) / ||r||; 3 u_i sqrt(n); 4..11 the static
// labels of the element (N(Q_l) / max(1, N), 2S_z(Q_l) / max(1, N), n(s)/2,
// n(t)/2, 2s_z(s), 2s_z(t), log(1 + m(Q_l)) / 8, (j + 0.5) / K).
// Training targets come from the converged vector psi of a step: at
// iteration k, t* = psi - (psi . u_k) u_k, alpha = (t* . dr) / (t* . t*)
// over the sampled elements (dr = d r), rho = alpha t* / dr and
// target = clamp(log rho, -3, 3) (rho > 0), -3 (rho <= 0), 0 (dr = 0).
// Loss: mean squared error; training: Adam (0.9, 0.999, 1e-8).
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include "core.h"

namespace dmrg {

constexpr int kMlpF = 12;
constexpr int kMlpH = 64;
constexpr int kMlpStatic = 8;
constexpr int kMlpP = kMlpH * kMlpF + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;  // 5057
constexpr int kMlpGradBlock = 64;  // elements per workgroup of the gradient kernel

// feat[i] = features of element e = idx ? idx[i] : i
void launch_mlp_features(const double* diag, const double* r, const double* u, const float* stat,
                         double theta, double rscale, double uscale, const int* idx, int64_t n_out,
                         float* feat, hipStream_t s);
void launch_mlp_forward(const float* params, const float* feat, int64_t n, float* out, hipStream_t s);
// t = r / (theta - diag) * exp(clamp(g, -3, 3))
void launch_mlp_precond(double* t, const double* r, const double* diag, double theta, const float* g,
                        int64_t n, hipStream_t s);
// dr[i] = r[e] / (theta - diag[e]), e = idx[i]
void launch_mlp_diag_corr(const double* r, const double* diag, double theta, const int* idx, int64_t n_out,
                          double* dr, hipStream_t s);
// per-workgroup partial gradients of sum_i (g_i - y_i)^2 / batch over the
// elements rows[0..n) (rows = idx ? idx[i] : i) of feat / y; partial is
// n_blocks x kMlpP, lossp n_blocks (sums of squared errors)
int64_t mlp_grad_blocks(int64_t n);
void launch_mlp_grad(const float* params, const float* feat, const float* y, const int* idx, int64_t n,
                     double batch, float* partial, float* lossp, hipStream_t s);
// grad[p] = sum_b partial[b][p] in block order; loss_out[0] = sum_b lossp[b]
void launch_mlp_reduce(const float* partial, const float* lossp, int64_t n_blocks, float* grad,
                       double* loss_out, hipStream_t s);
// Adam with bias-correction factors c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
void launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, float c1, float c2,
                     hipStream_t s);
// targets of one iteration at the sampled elements: psi, u full vectors,
// c = psi . u, dr sampled diagonal corrections
void launch_mlp_targets(const double* psi, const double* u, double c, const double* dr, const int* idx,
                        int64_t n_sample, float* target, hipStream_t s);

}  // namespace dmrg

namespace dmrg {

// counter-based generator (splitmix64) for initial weights, samples and
// epoch permutations
uint64_t splitmix64(uint64_t& state);

// Parameters, Adam moments and the collected training set on the device.
struct Mlp {
    hipStream_t s = nullptr;
    DevBuf params, m, v, grad, loss;
    DevBuf partial, lossp;  // gradient workspace
    int64_t step = 0;       // Adam steps taken
    DevBuf ds_x, ds_y;      // features (cap x 12) and targets (cap)
    int64_t ds_n = 0, ds_cap = 0;
    uint64_t seed = 0, draws = 0;
    std::mutex mu;  // append and draw_sample may be called from concurrent instances

    // params: host array of kMlpP values, or nullptr for the seeded
    // initialisation (uniform Glorot bounds, output layer scaled by 0.1,
    // zero biases)
    void init(hipStream_t st, const float* host_params, uint64_t seed_, int64_t capacity);
    // mean squared error over rows (idx ? idx[i] : i), i < n, of (feat, y);
    // gradient left in `grad`
    double loss_grad(const float* feat, const float* y, const int* idx, int64_t n);
    void adam(double lr);
    // append n device samples (features n x 12, targets n); returns how many fit
    int64_t append(const float* feat, const float* y, int64_t n);
    // epochs over the training set in seeded random order; mean batch loss of the last epoch
    double train(int epochs, int batch, double lr, uint64_t perm_seed);
    // sample indices for one Davidson step on a vector of n elements
    std::vector<int> draw_sample(int64_t n, int count);
};

}  // namespace dmrg
