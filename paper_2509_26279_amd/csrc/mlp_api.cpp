// Host side of the vetting MLP: parameters, buffers, seeded initialisation,
// training steps and inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

namespace sas {
void set_error(const std::string &msg);
}

using namespace sas;

struct sas_mlp {
    int64_t max_batch = 0;
    int64_t step = 0;
    uint64_t seed = 0;
    MlpBuffers b{};
    std::vector<void *> allocs;
};

namespace {

sas_status mfail(sas_status s, const std::string &m) {
    set_error(m);
    return s;
}

template <typename T>
bool dalloc(sas_mlp *m, T **p, size_t count) {
    void *d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    m->allocs.push_back(d);
    *p = (T *)d;
    return hipMemset(d, 0, std::max<size_t>(count, 1) * sizeof(T)) == hipSuccess;
}

uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

sas_status upload_params(sas_mlp *m, const float *host) {
    if (hipMemcpy(m->b.p, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->b.m, 0, sizeof(float) * kMlpParams) != hipSuccess ||
        hipMemset(m->b.v, 0, sizeof(float) * kMlpParams) != hipSuccess)
        return mfail(SAS_E_DEVICE, "sas_mlp: parameter upload");
    if (mlp_refresh(m->b, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return mfail(SAS_E_DEVICE, "sas_mlp: refreshing the bf16 weights");
    m->step = 0;
    return SAS_OK;
}

}  // namespace

extern "C" {

sas_status sas_mlp_create(int64_t max_batch, uint64_t seed, sas_mlp **out) {
    if (!out || max_batch < 1 || max_batch > ((int64_t)1 << 24))
        return mfail(SAS_E_INVALID, "sas_mlp_create: max_batch must be in [1, 2^24]");
    *out = nullptr;
    std::unique_ptr<sas_mlp> m(new sas_mlp());
    m->max_batch = max_batch;
    m->seed = seed;
    const size_t B = (size_t)max_batch, H = kMlpHidden;
    const size_t nz = (size_t)((max_batch + kMlpSplitK - 1) / kMlpSplitK);
    MlpBuffers &b = m->b;
    bool ok = dalloc(m.get(), &b.p, kMlpParams) && dalloc(m.get(), &b.m, kMlpParams) &&
              dalloc(m.get(), &b.v, kMlpParams) && dalloc(m.get(), &b.grad, kMlpParams) &&
              dalloc(m.get(), &b.w.w1, kMlpIn * H) && dalloc(m.get(), &b.w.w2, H * H) &&
              dalloc(m.get(), &b.w.w3, H * 16) && dalloc(m.get(), &b.w.b3pad, 16) &&
              dalloc(m.get(), &b.mu, kMlpIn) && dalloc(m.get(), &b.sd, kMlpIn) &&
              dalloc(m.get(), &b.a0, B * kMlpIn) && dalloc(m.get(), &b.h1, B * H) &&
              dalloc(m.get(), &b.h2, B * H) && dalloc(m.get(), &b.d1, B * H) &&
              dalloc(m.get(), &b.d2, B * H) && dalloc(m.get(), &b.z16, B * 16) &&
              dalloc(m.get(), &b.g3, B * 16) && dalloc(m.get(), &b.row_loss, B) &&
              dalloc(m.get(), &b.part, nz * H * H);
    if (!ok) {
        for (void *a : m->allocs) hipFree(a);
        return mfail(SAS_E_NOMEM, "sas_mlp_create: device memory");
    }
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a
    // counter-based generator seeded by `seed`.
    std::vector<float> p(kMlpParams, 0.0f);
    uint64_t st = seed;
    auto fill = [&](int off, int count, int fan_in) {
        const double bound = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < count; ++i) {
            const double u = (double)(splitmix64(&st) >> 11) * (1.0 / 9007199254740992.0);
            p[off + i] = (float)((2.0 * u - 1.0) * bound);
        }
    };
    fill(kMlpOffW1, kMlpIn * kMlpHidden, kMlpIn);
    fill(kMlpOffW2, kMlpHidden * kMlpHidden, kMlpHidden);
    fill(kMlpOffW3, kMlpHidden, kMlpHidden);
    std::vector<float> ones(kMlpIn, 1.0f);
    if (hipMemcpy(b.sd, ones.data(), sizeof(float) * kMlpIn, hipMemcpyHostToDevice) != hipSuccess) {
        for (void *a : m->allocs) hipFree(a);
        return mfail(SAS_E_DEVICE, "sas_mlp_create: upload");
    }
    sas_status s = upload_params(m.get(), p.data());
    if (s != SAS_OK) {
        for (void *a : m->allocs) hipFree(a);
        return s;
    }
    *out = m.release();
    return SAS_OK;
}

sas_status sas_mlp_destroy(sas_mlp *m) {
    if (!m) return SAS_OK;
    for (void *a : m->allocs) hipFree(a);
    delete m;
    return SAS_OK;
}

sas_status sas_mlp_set_norm(sas_mlp *m, const float *mean_host, const float *std_host) {
    if (!m || !mean_host || !std_host) return mfail(SAS_E_INVALID, "sas_mlp_set_norm: null argument");
    if (hipMemcpy(m->b.mu, mean_host, sizeof(float) * kMlpIn, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->b.sd, std_host, sizeof(float) * kMlpIn, hipMemcpyHostToDevice) != hipSuccess)
        return mfail(SAS_E_DEVICE, "sas_mlp_set_norm: upload");
    return SAS_OK;
}

sas_status sas_mlp_get_params(const sas_mlp *m, float *host, int64_t cap, int64_t *n_out) {
    if (!m || !n_out) return mfail(SAS_E_INVALID, "sas_mlp_get_params: null argument");
    *n_out = kMlpParams;
    if (cap < kMlpParams || !host) return mfail(SAS_E_OVERFLOW, "sas_mlp_get_params: cap < 20865");
    if (hipMemcpy(host, m->b.p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost) != hipSuccess)
        return mfail(SAS_E_DEVICE, "sas_mlp_get_params: copy");
    return SAS_OK;
}

sas_status sas_mlp_set_params(sas_mlp *m, const float *host, int64_t n) {
    if (!m || !host || n != kMlpParams)
        return mfail(SAS_E_INVALID, "sas_mlp_set_params: needs 20865 values");
    return upload_params(m, host);
}

// Checkpoint: a text header of kCkptHeader bytes (one JSON object, padded
// with spaces, ending in a newline), then float32 little-endian arrays:
// masters p, AdamW moments m and v (kMlpParams each), mean and std (kMlpIn
// each).  The header holds the format, the counts, the step and the seed.
constexpr int64_t kCkptHeader = 256;
constexpr int64_t kCkptFloats = 3 * (int64_t)kMlpParams + 2 * kMlpIn;
constexpr int64_t kCkptBytes = kCkptHeader + 4 * kCkptFloats;

sas_status sas_mlp_save(const sas_mlp *m, void *host, int64_t cap, int64_t *n_out) {
    if (!m || !n_out) return mfail(SAS_E_INVALID, "sas_mlp_save: null argument");
    *n_out = kCkptBytes;
    if (cap < kCkptBytes || !host)
        return mfail(SAS_E_OVERFLOW, "sas_mlp_save: cap below the checkpoint size in *n_out");
    char *out = (char *)host;
    std::string head = "{\"format\": \"sas_mlp\", \"version\": 1, \"params\": " +
                       std::to_string(kMlpParams) + ", \"inputs\": " + std::to_string(kMlpIn) +
                       ", \"step\": " + std::to_string(m->step) + ", \"seed\": " +
                       std::to_string(m->seed) +
                       ", \"layout\": \"float32 le: p, adam_m, adam_v, mean, std\"}";
    head.resize(kCkptHeader - 1, ' ');
    head.push_back('\n');
    std::memcpy(out, head.data(), kCkptHeader);
    float *f = (float *)(out + kCkptHeader);
    const struct {
        const float *src;
        int64_t n;
    } parts[] = {{m->b.p, kMlpParams}, {m->b.m, kMlpParams}, {m->b.v, kMlpParams},
                 {m->b.mu, kMlpIn}, {m->b.sd, kMlpIn}};
    for (const auto &pt : parts) {
        if (hipMemcpy(f, pt.src, sizeof(float) * pt.n, hipMemcpyDeviceToHost) != hipSuccess)
            return mfail(SAS_E_DEVICE, "sas_mlp_save: copy");
        f += pt.n;
    }
    return SAS_OK;
}

sas_status sas_mlp_load(sas_mlp *m, const void *host, int64_t n) {
    if (!m || !host) return mfail(SAS_E_INVALID, "sas_mlp_load: null argument");
    if (n != kCkptBytes) return mfail(SAS_E_INVALID, "sas_mlp_load: not a checkpoint of this size");
    const char *in = (const char *)host;
    const std::string head(in, kCkptHeader);
    long long step = -1, params = -1, inputs = -1, version = -1;
    unsigned long long seed = 0;
    const size_t ps = head.find("\"step\": "), pp = head.find("\"params\": "),
                 pi = head.find("\"inputs\": "), pv = head.find("\"version\": "),
                 pd = head.find("\"seed\": ");
    static const std::string kPrefix = "{\"format\": \"sas_mlp\",";
    if (head.compare(0, kPrefix.size(), kPrefix) != 0 || ps == std::string::npos ||
        pp == std::string::npos || pi == std::string::npos || pv == std::string::npos ||
        pd == std::string::npos || head.back() != '\n' ||
        std::sscanf(head.c_str() + ps + 8, "%lld", &step) != 1 ||
        std::sscanf(head.c_str() + pp + 10, "%lld", &params) != 1 ||
        std::sscanf(head.c_str() + pi + 10, "%lld", &inputs) != 1 ||
        std::sscanf(head.c_str() + pv + 11, "%lld", &version) != 1 ||
        std::sscanf(head.c_str() + pd + 8, "%llu", &seed) != 1)
        return mfail(SAS_E_INVALID, "sas_mlp_load: bad checkpoint header");
    if (version != 1 || params != kMlpParams || inputs != kMlpIn || step < 0)
        return mfail(SAS_E_INVALID, "sas_mlp_load: checkpoint of another network or version");
    const float *f = (const float *)(in + kCkptHeader);
    float *dst[] = {m->b.p, m->b.m, m->b.v, m->b.mu, m->b.sd};
    const int64_t cnt[] = {kMlpParams, kMlpParams, kMlpParams, kMlpIn, kMlpIn};
    for (int k = 0; k < 5; ++k) {
        if (hipMemcpy(dst[k], f, sizeof(float) * cnt[k], hipMemcpyHostToDevice) != hipSuccess)
            return mfail(SAS_E_DEVICE, "sas_mlp_load: upload");
        f += cnt[k];
    }
    if (mlp_refresh(m->b, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return mfail(SAS_E_DEVICE, "sas_mlp_load: refreshing the bf16 weights");
    m->step = step;
    m->seed = seed;
    return SAS_OK;
}

sas_status sas_mlp_forward(const sas_mlp *m, const float *x_dev, int64_t n, float *logits_dev,
                           void *stream) {
    if (!m || n < 0 || (n > 0 && (!x_dev || !logits_dev)))
        return mfail(SAS_E_INVALID, "sas_mlp_forward: bad argument");
    for (int64_t r0 = 0; r0 < n; r0 += m->max_batch) {
        const int64_t k = std::min(m->max_batch, n - r0);
        hipError_t e = mlp_logits(m->b, x_dev + r0 * kMlpIn, k, logits_dev + r0, (hipStream_t)stream);
        if (e != hipSuccess) return mfail(SAS_E_DEVICE, std::string("sas_mlp_forward: ") + hipGetErrorString(e));
    }
    return SAS_OK;
}

sas_status sas_mlp_grad(const sas_mlp *m, const float *x_dev, const float *y_dev, int64_t batch,
                        float pos_weight, float *loss_dev, float *grad_dev, void *stream) {
    if (!m || batch < 1 || batch > m->max_batch || !x_dev || !y_dev || !loss_dev || !grad_dev)
        return mfail(SAS_E_INVALID, "sas_mlp_grad: bad argument (batch in [1, max_batch])");
    hipError_t e = mlp_grad(m->b, x_dev, y_dev, batch, pos_weight, loss_dev, grad_dev,
                            (hipStream_t)stream);
    if (e != hipSuccess) return mfail(SAS_E_DEVICE, std::string("sas_mlp_grad: ") + hipGetErrorString(e));
    return SAS_OK;
}

sas_status sas_mlp_train_step(sas_mlp *m, const float *x_dev, const float *y_dev, int64_t batch,
                              float pos_weight, float lr, float beta1, float beta2, float eps,
                              float weight_decay, float *loss_dev, void *stream) {
    if (!m || batch < 1 || batch > m->max_batch || !x_dev || !y_dev || !loss_dev)
        return mfail(SAS_E_INVALID, "sas_mlp_train_step: bad argument (batch in [1, max_batch])");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = mlp_grad(m->b, x_dev, y_dev, batch, pos_weight, loss_dev, m->b.grad, s);
    if (e != hipSuccess) return mfail(SAS_E_DEVICE, std::string("sas_mlp_train_step: ") + hipGetErrorString(e));
    m->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)m->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)m->step));
    e = mlp_adamw(m->b, m->b.grad, lr, beta1, beta2, eps, weight_decay, (float)c1, (float)c2, s);
    if (e != hipSuccess) return mfail(SAS_E_DEVICE, std::string("sas_mlp_train_step: ") + hipGetErrorString(e));
    return SAS_OK;
}

}  // extern "C"
