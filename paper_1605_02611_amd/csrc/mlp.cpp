// Host side of the learned Davidson preconditioner: parameters, Adam,
// training set and training loop (kernels in mlp.hip).
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace dmrg {

uint64_t splitmix64(uint64_t& state) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t& st) { return double(splitmix64(st) >> 11) * 0x1p-53; }

void Mlp::init(hipStream_t st, const float* host_params, uint64_t seed_, int64_t capacity) {
    s = st;
    seed = seed_;
    std::vector<float> h(kMlpP, 0.0f);
    if (host_params) {
        std::copy(host_params, host_params + kMlpP, h.begin());
        for (float x : h) require(std::isfinite(x), "MLP parameters must be finite");
    } else {
        uint64_t g = seed;
        auto fill = [&](int off, int count, double bound) {
            for (int i = 0; i < count; ++i) h[off + i] = float((2.0 * uniform01(g) - 1.0) * bound);
        };
        const int oB1 = kMlpH * kMlpF, oW2 = oB1 + kMlpH, oB2 = oW2 + kMlpH * kMlpH, oW3 = oB2 + kMlpH;
        fill(0, kMlpH * kMlpF, std::sqrt(6.0 / (kMlpF + kMlpH)));
        fill(oW2, kMlpH * kMlpH, std::sqrt(6.0 / (2 * kMlpH)));
        fill(oW3, kMlpH, 0.1 * std::sqrt(6.0 / (kMlpH + 1)));
    }
    params.alloc(kMlpP * sizeof(float), s);
    m.alloc(kMlpP * sizeof(float), s);
    v.alloc(kMlpP * sizeof(float), s);
    grad.alloc(kMlpP * sizeof(float), s);
    loss.alloc(sizeof(double), s);
    DMRG_HIP(hipMemcpyAsync(params.p, h.data(), kMlpP * sizeof(float), hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemsetAsync(m.p, 0, m.bytes, s));
    DMRG_HIP(hipMemsetAsync(v.p, 0, v.bytes, s));
    step = 0;
    ds_cap = std::max<int64_t>(0, capacity);
    ds_n = 0;
    if (ds_cap > 0) {
        ds_x.alloc(size_t(ds_cap) * kMlpF * sizeof(float), s);
        ds_y.alloc(size_t(ds_cap) * sizeof(float), s);
    }
    DMRG_HIP(hipStreamSynchronize(s));
}

double Mlp::loss_grad(const float* feat, const float* y, const int* idx, int64_t n) {
    require(n >= 1, "MLP loss: empty batch");
    const int64_t nb = mlp_grad_blocks(n);
    if (int64_t(partial.bytes) < nb * kMlpP * int64_t(sizeof(float))) {
        partial.alloc(size_t(nb) * kMlpP * sizeof(float), s);
        lossp.alloc(size_t(nb) * sizeof(float), s);
    }
    launch_mlp_grad(params.as<float>(), feat, y, idx, n, double(n), partial.as<float>(), lossp.as<float>(), s);
    launch_mlp_reduce(partial.as<float>(), lossp.as<float>(), nb, grad.as<float>(), loss.as<double>(), s);
    double h = 0;
    DMRG_HIP(hipMemcpyAsync(&h, loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return h / double(n);
}

void Mlp::adam(double lr) {
    ++step;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, double(step)));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, double(step)));
    launch_mlp_adam(params.as<float>(), m.as<float>(), v.as<float>(), grad.as<float>(), float(lr), float(c1),
                    float(c2), s);
}

int64_t Mlp::append(const float* feat, const float* y, int64_t n) {
    std::lock_guard<std::mutex> lk(mu);
    const int64_t k = std::min(n, ds_cap - ds_n);
    if (k <= 0) return 0;
    DMRG_HIP(hipMemcpyAsync(ds_x.as<float>() + ds_n * kMlpF, feat, size_t(k) * kMlpF * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    DMRG_HIP(hipMemcpyAsync(ds_y.as<float>() + ds_n, y, size_t(k) * sizeof(float), hipMemcpyDeviceToDevice, s));
    ds_n += k;
    DMRG_HIP(hipStreamSynchronize(s));
    return k;
}

double Mlp::train(int epochs, int batch, double lr, uint64_t perm_seed) {
    require(epochs >= 1 && batch >= 1 && lr > 0, "MLP training: invalid options");
    require(ds_n >= 1, "MLP training: the training set is empty", E_STATE);
    std::vector<int> perm(ds_n);
    DevBuf dperm(size_t(ds_n) * sizeof(int), s);
    double last = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        uint64_t g = perm_seed + 0x632be59bd9b4e019ULL * uint64_t(ep + 1);
        for (int64_t i = ds_n - 1; i > 0; --i) {
            const int64_t j = int64_t(splitmix64(g) % uint64_t(i + 1));
            std::swap(perm[i], perm[j]);
        }
        DMRG_HIP(hipMemcpyAsync(dperm.p, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, s));
        double sum = 0;
        int nbat = 0;
        for (int64_t b0 = 0; b0 < ds_n; b0 += batch) {
            const int64_t nb = std::min<int64_t>(batch, ds_n - b0);
            sum += loss_grad(ds_x.as<float>(), ds_y.as<float>(), dperm.as<int>() + b0, nb);
            adam(lr);
            ++nbat;
        }
        last = sum / std::max(1, nbat);
    }
    DMRG_HIP(hipStreamSynchronize(s));
    return last;
}

std::vector<int> Mlp::draw_sample(int64_t n, int count) {
    std::lock_guard<std::mutex> lk(mu);
    std::vector<int> idx(std::max(0, count));
    uint64_t g = seed ^ (0xd1b54a32d192ed03ULL * (++draws));
    for (int& i : idx) i = int(splitmix64(g) % uint64_t(n));
    return idx;
}

}  // namespace dmrg
