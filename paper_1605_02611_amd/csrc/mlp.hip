// Kernels of the learned Davidson preconditioner (gfx950): features,
// inference, the learned correction, training gradients with a fixed-order
// reduction, Adam, and the training targets.  Definitions in mlp.h.
#include <hip/hip_runtime.h>

#include "mlp.h"

namespace dmrg {

namespace {

constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kMlpH * kMlpF;
constexpr int oW2 = oB1 + kMlpH;
constexpr int oB2 = oW2 + kMlpH * kMlpH;
constexpr int oW3 = oB2 + kMlpH;
constexpr int oB3 = oW3 + kMlpH;
static_assert(oB3 + 1 == kMlpP, "parameter layout");

__device__ inline double clamp_den(double den) {
    if (fabs(den) < 1e-12) den = den < 0 ? -1e-12 : 1e-12;
    return den;
}

inline unsigned grid_of(int64_t n, int block = 256, int cap = 16384) {
    int64_t g = (n + block - 1) / block;
    return unsigned(g < 1 ? 1 : (g > cap ? cap : g));
}

__global__ void features_kernel(const double* __restrict__ diag, const double* __restrict__ r,
                                const double* __restrict__ u, const float* __restrict__ stat, double theta,
                                double inv_se, double rscale, double uscale, const int* __restrict__ idx,
                                int64_t n_out, float* __restrict__ feat) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_out;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t e = idx ? idx[i] : i;
        const double den = theta - diag[e];
        float* f = feat + i * kMlpF;
        f[0] = float(den * inv_se);
        f[1] = float(log(fmax(fabs(den), 1e-12)) / 10.0);
        f[2] = float(r[e] * rscale);
        f[3] = float(u[e] * uscale);
        for (int c = 0; c < kMlpStatic; ++c) f[4 + c] = stat[e * kMlpStatic + c];
    }
}

// one element per thread; parameters in LDS, read as broadcasts
__global__ __launch_bounds__(256) void forward_kernel(const float* __restrict__ params,
                                                      const float* __restrict__ feat, int64_t n,
                                                      float* __restrict__ out) {
    __shared__ float w[kMlpP];
    for (int p = threadIdx.x; p < kMlpP; p += blockDim.x) w[p] = params[p];
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        float x[kMlpF];
#pragma unroll
        for (int c = 0; c < kMlpF; ++c) x[c] = feat[i * kMlpF + c];
        // fully unrolled over the hidden index so that h1 stays in registers
        float h1[kMlpH];
#pragma unroll
        for (int j = 0; j < kMlpH; ++j) {
            float z = w[oB1 + j];
#pragma unroll
            for (int c = 0; c < kMlpF; ++c) z = fmaf(w[oW1 + j * kMlpF + c], x[c], z);
            h1[j] = tanhf(z);
        }
        float g = w[oB3];
        for (int j = 0; j < kMlpH; ++j) {
            float z = w[oB2 + j];
#pragma unroll
            for (int k = 0; k < kMlpH; ++k) z = fmaf(w[oW2 + j * kMlpH + k], h1[k], z);
            g = fmaf(w[oW3 + j], tanhf(z), g);
        }
        out[i] = g;
    }
}

__global__ void precond_kernel(double* __restrict__ t, const double* __restrict__ r,
                               const double* __restrict__ diag, double theta, const float* __restrict__ g,
                               int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        const double gc = fmin(3.0, fmax(-3.0, double(g[e])));
        t[e] = r[e] / clamp_den(theta - diag[e]) * exp(gc);
    }
}

__global__ void diag_corr_kernel(const double* __restrict__ r, const double* __restrict__ diag, double theta,
                                 const int* __restrict__ idx, int64_t n_out, double* __restrict__ dr) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_out;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t e = idx[i];
        dr[i] = r[e] / clamp_den(theta - diag[e]);
    }
}

// One workgroup of kMlpGradBlock threads = kMlpGradBlock elements: forward
// and backward per element into LDS, then every parameter's gradient summed
// over the block's elements in element order (deterministic).
__global__ __launch_bounds__(kMlpGradBlock) void grad_kernel(const float* __restrict__ params,
                                                             const float* __restrict__ feat,
                                                             const float* __restrict__ y,
                                                             const int* __restrict__ idx, int64_t n,
                                                             float inv_batch, float* __restrict__ partial,
                                                             float* __restrict__ lossp) {
    constexpr int B = kMlpGradBlock;
    __shared__ float w[kMlpP];
    __shared__ float X[B][kMlpF];
    __shared__ float H1[B][kMlpH + 1];
    __shared__ float DZ1[B][kMlpH + 1];
    __shared__ float DZ2[B][kMlpH + 1];
    __shared__ float G3[B][kMlpH + 1];
    __shared__ float DG[B];
    __shared__ float E2[B];
    const int t = threadIdx.x;
    for (int p = t; p < kMlpP; p += B) w[p] = params[p];
    const int64_t i = int64_t(blockIdx.x) * B + t;
    const bool live = i < n;
    const int64_t row = live ? (idx ? int64_t(idx[i]) : i) : 0;
    for (int c = 0; c < kMlpF; ++c) X[t][c] = live ? feat[row * kMlpF + c] : 0.0f;
    __syncthreads();
    // forward
    for (int j = 0; j < kMlpH; ++j) {
        float z = w[oB1 + j];
        for (int c = 0; c < kMlpF; ++c) z = fmaf(w[oW1 + j * kMlpF + c], X[t][c], z);
        H1[t][j] = tanhf(z);
    }
    float h2[kMlpH];
    float g = w[oB3];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float z = w[oB2 + j];
        for (int k = 0; k < kMlpH; ++k) z = fmaf(w[oW2 + j * kMlpH + k], H1[t][k], z);
        h2[j] = tanhf(z);
        g = fmaf(w[oW3 + j], h2[j], g);
    }
    // backward of (g - y)^2 / batch
    const float e = live ? g - y[row] : 0.0f;
    const float dg = 2.0f * e * inv_batch;
    DG[t] = dg;
    E2[t] = e * e;
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        G3[t][j] = dg * h2[j];
        DZ2[t][j] = dg * w[oW3 + j] * (1.0f - h2[j] * h2[j]);
    }
    for (int k = 0; k < kMlpH; ++k) {
        float s = 0.0f;
        for (int j = 0; j < kMlpH; ++j) s = fmaf(DZ2[t][j], w[oW2 + j * kMlpH + k], s);
        const float h = H1[t][k];
        DZ1[t][k] = s * (1.0f - h * h);
    }
    __syncthreads();
    float* out = partial + int64_t(blockIdx.x) * kMlpP;
    for (int p = t; p < kMlpP; p += B) {
        float s = 0.0f;
        if (p < oB1) {
            const int j = p / kMlpF, c = p % kMlpF;
            for (int a = 0; a < B; ++a) s = fmaf(DZ1[a][j], X[a][c], s);
        } else if (p < oW2) {
            const int j = p - oB1;
            for (int a = 0; a < B; ++a) s += DZ1[a][j];
        } else if (p < oB2) {
            const int q = p - oW2, j = q / kMlpH, k = q % kMlpH;
            for (int a = 0; a < B; ++a) s = fmaf(DZ2[a][j], H1[a][k], s);
        } else if (p < oW3) {
            const int j = p - oB2;
            for (int a = 0; a < B; ++a) s += DZ2[a][j];
        } else if (p < oB3) {
            const int j = p - oW3;
            for (int a = 0; a < B; ++a) s += G3[a][j];
        } else {
            for (int a = 0; a < B; ++a) s += DG[a];
        }
        out[p] = s;
    }
    if (t == 0) {
        float s = 0.0f;
        for (int a = 0; a < B; ++a) s += E2[a];
        lossp[blockIdx.x] = s;
    }
}

__global__ void reduce_kernel(const float* __restrict__ partial, const float* __restrict__ lossp,
                              int64_t n_blocks, float* __restrict__ grad, double* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpP) {
        float s = 0.0f;
        for (int64_t b = 0; b < n_blocks; ++b) s += partial[b * kMlpP + p];
        grad[p] = s;
    }
    if (p == 0) {
        double s = 0.0;
        for (int64_t b = 0; b < n_blocks; ++b) s += double(lossp[b]);
        *loss_out = s;
    }
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float lr, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpP) return;
    const float gp = g[p];
    const float mp = 0.9f * m[p] + 0.1f * gp;
    const float vp = 0.999f * v[p] + 0.001f * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + 1e-8f);
}

// one workgroup: alpha from fixed-order partial sums, then the targets
__global__ __launch_bounds__(256) void targets_kernel(const double* __restrict__ psi, const double* __restrict__ u,
                                                      double c, const double* __restrict__ dr,
                                                      const int* __restrict__ idx, int64_t ns,
                                                      float* __restrict__ target) {
    __shared__ double sa[256], sb[256];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = t; i < ns; i += 256) {
        const int64_t e = idx[i];
        const double ts = psi[e] - c * u[e];
        a += ts * dr[i];
        b += ts * ts;
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    const double alpha = sb[0] > 0 ? sa[0] / sb[0] : 0.0;
    for (int64_t i = t; i < ns; i += 256) {
        const int64_t e = idx[i];
        const double d = dr[i];
        float out = 0.0f;
        if (d != 0.0) {
            const double rho = alpha * (psi[e] - c * u[e]) / d;
            out = rho > 0 ? float(fmin(3.0, fmax(-3.0, log(rho)))) : -3.0f;
        }
        target[i] = out;
    }
}

}  // namespace

void launch_mlp_features(const double* diag, const double* r, const double* u, const float* stat,
                         double theta, double rscale, double uscale, const int* idx, int64_t n_out,
                         float* feat, hipStream_t s) {
    if (n_out <= 0) return;
    hipLaunchKernelGGL(features_kernel, dim3(grid_of(n_out)), dim3(256), 0, s, diag, r, u, stat, theta,
                       1.0 / fmax(1.0, fabs(theta)), rscale, uscale, idx, n_out, feat);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_forward(const float* params, const float* feat, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(forward_kernel, dim3(grid_of(n, 256, 4096)), dim3(256), 0, s, params, feat, n, out);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_precond(double* t, const double* r, const double* diag, double theta, const float* g,
                        int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(precond_kernel, dim3(grid_of(n)), dim3(256), 0, s, t, r, diag, theta, g, n);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_diag_corr(const double* r, const double* diag, double theta, const int* idx, int64_t n_out,
                          double* dr, hipStream_t s) {
    if (n_out <= 0) return;
    hipLaunchKernelGGL(diag_corr_kernel, dim3(grid_of(n_out)), dim3(256), 0, s, r, diag, theta, idx, n_out, dr);
    DMRG_HIP(hipGetLastError());
}

int64_t mlp_grad_blocks(int64_t n) { return (n + kMlpGradBlock - 1) / kMlpGradBlock; }

void launch_mlp_grad(const float* params, const float* feat, const float* y, const int* idx, int64_t n,
                     double batch, float* partial, float* lossp, hipStream_t s) {
    const int64_t nb = mlp_grad_blocks(n);
    require(nb >= 1 && nb < (int64_t(1) << 31), "MLP gradient: bad batch size");
    hipLaunchKernelGGL(grad_kernel, dim3(unsigned(nb)), dim3(kMlpGradBlock), 0, s, params, feat, y, idx, n,
                       float(1.0 / batch), partial, lossp);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_reduce(const float* partial, const float* lossp, int64_t n_blocks, float* grad,
                       double* loss_out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3((kMlpP + 255) / 256), dim3(256), 0, s, partial, lossp, n_blocks,
                       grad, loss_out);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, float c1, float c2,
                     hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpP + 255) / 256), dim3(256), 0, s, params, m, v, grad, lr, c1, c2);
    DMRG_HIP(hipGetLastError());
}

void launch_mlp_targets(const double* psi, const double* u, double c, const double* dr, const int* idx,
                        int64_t n_sample, float* target, hipStream_t s) {
    if (n_sample <= 0) return;
    hipLaunchKernelGGL(targets_kernel, dim3(1), dim3(256), 0, s, psi, u, c, dr, idx, n_sample, target);
    DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
