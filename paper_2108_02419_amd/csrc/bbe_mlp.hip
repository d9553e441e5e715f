// bbe_mlp.hip -- C ABI of the surrogate network (include/bbe.h): device
// buffers, the training step as a fixed kernel sequence, the encoder.
#include "abi_internal.hpp"
#include "mlp.hpp"

#include <cmath>
#include <new>
#include <vector>

using namespace bbe_abi;

struct bbe_mlp {
    int max_batch = 0;
    long step = 0;
    float* params = nullptr;  // fp32 master [kNParams]
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    uint16_t *w1 = nullptr, *w2 = nullptr, *w3 = nullptr, *w4 = nullptr;
    uint16_t *w2t = nullptr, *w3t = nullptr, *w4t = nullptr;
    uint16_t *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    uint16_t *dz4 = nullptr, *dz3 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    bbe::WgradTile* tiles = nullptr;
    int n_tiles = 0;
    float* wpart = nullptr;  // [chunks of kWgRows rows][kNParams], when max_batch > kWgRows
};

namespace {

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;

void destroy(bbe_mlp* m) {
    if (!m) return;
    if (m->params) (void)hipDeviceSynchronize();
    void* ptrs[] = {m->params, m->m,   m->v,   m->grad, m->w1,  m->w2,  m->w3,  m->w4,
                    m->w2t,    m->w3t, m->w4t, m->h1,   m->h2,  m->h3,  m->dz4, m->dz3,
                    m->dz2,    m->dz1, m->tiles, m->wpart};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

template <typename T>
bool alloc(T** p, size_t count) {
    return dev_alloc(p, count * sizeof(T)) == hipSuccess;
}

bbe::MlpAdamArgs adam_args(bbe_mlp* m, const float* grad, float lr) {
    bbe::MlpAdamArgs a;
    a.params = m->params;
    a.m = m->m;
    a.v = m->v;
    a.grad = grad;
    a.lr = lr;
    a.beta1 = kBeta1;
    a.beta2 = kBeta2;
    a.eps = kEps;
    const double t = (double)(m->step > 0 ? m->step : 1);
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)kBeta1, t)));
    a.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)kBeta2, t)));
    a.w1 = m->w1;
    a.w2 = m->w2;
    a.w3 = m->w3;
    a.w4 = m->w4;
    a.w2t = m->w2t;
    a.w3t = m->w3t;
    a.w4t = m->w4t;
    return a;
}

bbe::MlpFwdArgs fwd_args(const bbe_mlp* m, const uint16_t* x, const int32_t* nv, int B) {
    bbe::MlpFwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = x;
    a.n_valid = nv;
    a.B = B;
    a.w1 = m->w1;
    a.w2 = m->w2;
    a.w3 = m->w3;
    a.w4 = m->w4;
    a.b1 = m->params + bbe::kOffB1;
    a.b2 = m->params + bbe::kOffB2;
    a.b3 = m->params + bbe::kOffB3;
    a.b4 = m->params + bbe::kOffB4;
    a.inv_batch = 1.0f / (float)B;
    return a;
}

}  // namespace

BBE_API int bbe_mlp_create(const float* params, int max_batch, bbe_mlp** out) {
    if (!out) return fail(BBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params) return fail(BBE_EINVAL, "params is NULL");
    if (max_batch < 1) return fail(BBE_EINVAL, "max_batch must be >= 1");
    for (int i = 0; i < bbe::kNParams; ++i)
        if (!std::isfinite(params[i])) return fail(BBE_EINVAL, "params[%d] is not finite", i);
    bbe_mlp* m = new (std::nothrow) bbe_mlp();
    if (!m) return fail(BBE_ENOMEM, "out of host memory");
    m->max_batch = max_batch;
    const size_t B = (size_t)max_batch;
    bool okk = alloc(&m->params, bbe::kNParams) && alloc(&m->m, bbe::kNParams) &&
               alloc(&m->v, bbe::kNParams) && alloc(&m->grad, bbe::kNParams) &&
               alloc(&m->w1, (size_t)bbe::kHid * bbe::kIn) &&
               alloc(&m->w2, (size_t)bbe::kHid * bbe::kHid) &&
               alloc(&m->w3, (size_t)bbe::kHid * bbe::kHid) &&
               alloc(&m->w4, (size_t)bbe::kOutP * bbe::kHid) &&
               alloc(&m->w2t, (size_t)bbe::kHid * bbe::kHid) &&
               alloc(&m->w3t, (size_t)bbe::kHid * bbe::kHid) &&
               alloc(&m->w4t, (size_t)bbe::kHid * bbe::kOutP) &&
               alloc(&m->h1, B * bbe::kHid) && alloc(&m->h2, B * bbe::kHid) &&
               alloc(&m->h3, B * bbe::kHid) && alloc(&m->dz4, B * bbe::kOutP) &&
               alloc(&m->dz3, B * bbe::kHid) && alloc(&m->dz2, B * bbe::kHid) &&
               alloc(&m->dz1, B * bbe::kHid);
    // weight-gradient work tiles: 64 x 64 blocks of each layer
    std::vector<bbe::WgradTile> tiles;
    const int rows[4] = {bbe::kHid, bbe::kHid, bbe::kHid, bbe::kOut};
    const int ks[4] = {bbe::kIn, bbe::kHid, bbe::kHid, bbe::kHid};
    for (int l = 0; l < 4; ++l)
        for (int n0 = 0; n0 < rows[l]; n0 += 64)
            for (int k0 = 0; k0 < ks[l]; k0 += 64) tiles.push_back({l, n0, k0, 0});
    m->n_tiles = (int)tiles.size();
    okk = okk && alloc(&m->tiles, tiles.size());
    const size_t chunks = (B + bbe::kWgRows - 1) / bbe::kWgRows;
    if (chunks > 1) okk = okk && alloc(&m->wpart, chunks * bbe::kNParams);
    if (!okk) {
        destroy(m);
        return fail(BBE_ENOMEM, "device allocation of the network failed");
    }
    hipError_t e = BBE_HIP(hipMemcpy(m->params, params, sizeof(float) * bbe::kNParams,
                                     hipMemcpyHostToDevice));
    if (e == hipSuccess)
        e = hipMemcpy(m->tiles, tiles.data(), sizeof(bbe::WgradTile) * tiles.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->m, 0, sizeof(float) * bbe::kNParams);
    if (e == hipSuccess) e = hipMemset(m->v, 0, sizeof(float) * bbe::kNParams);
    // padding rows / columns of the last layer's copies stay zero
    if (e == hipSuccess) e = hipMemset(m->w4, 0, sizeof(uint16_t) * bbe::kOutP * bbe::kHid);
    if (e == hipSuccess) e = hipMemset(m->w4t, 0, sizeof(uint16_t) * bbe::kHid * bbe::kOutP);
    if (e == hipSuccess) e = bbe::launch_mlp_adam(adam_args(m, nullptr, 0.0f), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy(m);
        return hip_fail(e, "initialising the network");
    }
    *out = m;
    return ok();
}

BBE_API void bbe_mlp_free(bbe_mlp* m) { destroy(m); }

BBE_API int bbe_mlp_get_params(const bbe_mlp* m, float* params) {
    if (!m || !params) return fail(BBE_EINVAL, "NULL argument");
    hipError_t e = hipMemcpy(params, m->params, sizeof(float) * bbe::kNParams,
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copying the parameters");
    return ok();
}

// File layouts (little endian): parameters only -- 8-byte magic
// "BBEMLP01", uint32 parameter count, the float32 master parameters in the
// packing of BBE_MLP_NPARAMS; training checkpoint -- magic "BBEMLP02",
// uint32 parameter count, uint64 Adam steps taken, then parameters, Adam
// first moments and Adam second moments (float32, same packing).
static const char kMagic[8] = {'B', 'B', 'E', 'M', 'L', 'P', '0', '1'};
static const char kMagicCkpt[8] = {'B', 'B', 'E', 'M', 'L', 'P', '0', '2'};

BBE_API int bbe_mlp_save(const bbe_mlp* m, const char* path) {
    if (!m || !path) return fail(BBE_EINVAL, "NULL argument");
    std::vector<float> p((size_t)bbe::kNParams);
    int rc = bbe_mlp_get_params(m, p.data());
    if (rc != BBE_OK) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(BBE_EINVAL, "cannot open %s for writing", path);
    const uint32_t count = (uint32_t)bbe::kNParams;
    bool good = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
                std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    good = (std::fclose(f) == 0) && good;
    if (!good) return fail(BBE_EINVAL, "writing %s failed", path);
    return ok();
}

BBE_API int bbe_mlp_save_checkpoint(const bbe_mlp* m, const char* path) {
    if (!m || !path) return fail(BBE_EINVAL, "NULL argument");
    const size_t np = (size_t)bbe::kNParams;
    std::vector<float> buf(3 * np);
    const float* src[3] = {m->params, m->m, m->v};
    for (int i = 0; i < 3; ++i) {
        hipError_t e = BBE_HIP(hipMemcpy(buf.data() + i * np, src[i], sizeof(float) * np,
                                         hipMemcpyDeviceToHost));
        if (e != hipSuccess) return hip_fail(e, "copying the training state");
    }
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(BBE_EINVAL, "cannot open %s for writing", path);
    const uint32_t count = (uint32_t)bbe::kNParams;
    const uint64_t step = (uint64_t)m->step;
    bool good = std::fwrite(kMagicCkpt, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
                std::fwrite(&step, 8, 1, f) == 1 &&
                std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    good = (std::fclose(f) == 0) && good;
    if (!good) return fail(BBE_EINVAL, "writing %s failed", path);
    return ok();
}

BBE_API int bbe_mlp_load(const char* path, int max_batch, bbe_mlp** out) {
    if (!out) return fail(BBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!path) return fail(BBE_EINVAL, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(BBE_EINVAL, "cannot open %s", path);
    char magic[8];
    uint32_t count = 0;
    uint64_t step = 0;
    const size_t np = (size_t)bbe::kNParams;
    bool good = std::fread(magic, 1, 8, f) == 8;
    const bool ckpt = good && std::memcmp(magic, kMagicCkpt, 8) == 0;
    good = good && (ckpt || std::memcmp(magic, kMagic, 8) == 0) &&
           std::fread(&count, 4, 1, f) == 1 && count == (uint32_t)bbe::kNParams;
    if (good && ckpt) good = std::fread(&step, 8, 1, f) == 1;
    std::vector<float> p((ckpt ? 3 : 1) * np);
    good = good && std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    char extra;
    good = good && std::fread(&extra, 1, 1, f) == 0;  // nothing after the data
    std::fclose(f);
    if (!good) return fail(BBE_EINVAL, "%s is not a saved network of %d parameters", path,
                           bbe::kNParams);
    if (ckpt)
        for (size_t i = np; i < 3 * np; ++i)
            if (!std::isfinite(p[i]) || (i >= 2 * np && p[i] < 0.0f))
                return fail(BBE_EINVAL, "%s: Adam moment %zu is not valid", path, i - np);
    bbe_mlp* m = nullptr;
    int rc = bbe_mlp_create(p.data(), max_batch, &m);
    if (rc != BBE_OK) return rc;
    if (ckpt) {
        hipError_t e = BBE_HIP(hipMemcpy(m->m, p.data() + np, sizeof(float) * np,
                                         hipMemcpyHostToDevice));
        if (e == hipSuccess)
            e = hipMemcpy(m->v, p.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            destroy(m);
            return hip_fail(e, "restoring the Adam state");
        }
        m->step = (long)step;
    }
    *out = m;
    return ok();
}

BBE_API int bbe_mlp_forward(const bbe_mlp* m, const uint16_t* x, const int32_t* n_valid,
                            int batch, float* probs, float* entropy, float* logits,
                            void* stream) {
    if (!m || !x || !n_valid) return fail(BBE_EINVAL, "NULL argument");
    if (batch < 1) return fail(BBE_EINVAL, "batch must be >= 1");
    bbe::MlpFwdArgs a = fwd_args(m, x, n_valid, batch);
    a.probs = probs;
    a.entropy = entropy;
    a.logits = logits;
    hipError_t e = BBE_HIP(bbe::launch_mlp_fwd(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching the forward pass");
    return ok();
}

BBE_API int bbe_mlp_forward_hidden(const bbe_mlp* m, const uint16_t* x, const int32_t* n_valid,
                                   int batch, uint16_t* hidden, float* logits, void* stream) {
    if (!m || !x || !n_valid || !hidden) return fail(BBE_EINVAL, "NULL argument");
    if (batch < 1) return fail(BBE_EINVAL, "batch must be >= 1");
    bbe::MlpFwdArgs a = fwd_args(m, x, n_valid, batch);
    const size_t layer = (size_t)batch * bbe::kHid;
    a.h1 = hidden;
    a.h2 = hidden + layer;
    a.h3 = hidden + 2 * layer;
    a.logits = logits;
    hipError_t e = BBE_HIP(bbe::launch_mlp_fwd(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching the forward pass");
    return ok();
}

BBE_API int bbe_mlp_loss_grad(bbe_mlp* m, const uint16_t* x, const int32_t* n_valid,
                              const float* target, int batch, float* loss, float* grad,
                              void* stream) {
    if (!m || !x || !n_valid || !target || !loss) return fail(BBE_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->max_batch)
        return fail(BBE_EINVAL, "batch must be in 1..%d", m->max_batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* g = grad ? grad : m->grad;
    hipError_t e = BBE_HIP(bbe::launch_fill_f32(loss, 0.0f, 1, s));
    if (e == hipSuccess) e = bbe::launch_fill_f32(g, 0.0f, bbe::kNParams, s);
    bbe::MlpFwdArgs f = fwd_args(m, x, n_valid, batch);
    f.h1 = m->h1;
    f.h2 = m->h2;
    f.h3 = m->h3;
    f.target = target;
    f.dz = m->dz4;
    f.loss = loss;
    if (e == hipSuccess) e = bbe::launch_mlp_fwd(f, s);
    bbe::MlpBwdArgs b;
    b.B = batch;
    b.dz4 = m->dz4;
    b.w4t = m->w4t;
    b.w3t = m->w3t;
    b.w2t = m->w2t;
    b.h1 = m->h1;
    b.h2 = m->h2;
    b.h3 = m->h3;
    b.dz3 = m->dz3;
    b.dz2 = m->dz2;
    b.dz1 = m->dz1;
    if (e == hipSuccess) e = bbe::launch_mlp_bwd_data(b, s);
    bbe::MlpWgradArgs w;
    w.B = batch;
    w.tiles = m->tiles;
    w.layers[0] = {m->dz1, bbe::kHid, x, bbe::kIn, bbe::kHid, g + bbe::kOffW1, g + bbe::kOffB1,
                   bbe::kOffW1};
    w.layers[1] = {m->dz2, bbe::kHid, m->h1, bbe::kHid, bbe::kHid, g + bbe::kOffW2,
                   g + bbe::kOffB2, bbe::kOffW2};
    w.layers[2] = {m->dz3, bbe::kHid, m->h2, bbe::kHid, bbe::kHid, g + bbe::kOffW3,
                   g + bbe::kOffB3, bbe::kOffW3};
    w.layers[3] = {m->dz4, bbe::kOutP, m->h3, bbe::kHid, bbe::kOut, g + bbe::kOffW4,
                   g + bbe::kOffB4, bbe::kOffW4};
    w.part = m->wpart;
    if (e == hipSuccess) e = bbe::launch_mlp_wgrad(w, m->n_tiles, s);
    if (e != hipSuccess) return hip_fail(e, "launching the backward pass");
    return ok();
}

BBE_API int bbe_mlp_adam_step(bbe_mlp* m, const float* grad, float lr, void* stream) {
    if (!m) return fail(BBE_EINVAL, "NULL network");
    if (!std::isfinite(lr) || !(lr > 0.0f)) return fail(BBE_EINVAL, "lr must be finite and > 0");
    m->step += 1;
    hipError_t e = BBE_HIP(bbe::launch_mlp_adam(adam_args(m, grad ? grad : m->grad, lr),
                                        static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching the Adam step");
    return ok();
}

BBE_API int bbe_mlp_train_step(bbe_mlp* m, const uint16_t* x, const int32_t* n_valid,
                               const float* target, int batch, float lr, float* loss,
                               void* stream) {
    int rc = bbe_mlp_loss_grad(m, x, n_valid, target, batch, loss, nullptr, stream);
    if (rc != BBE_OK) return rc;
    return bbe_mlp_adam_step(m, nullptr, lr, stream);
}

BBE_API int bbe_encode_states(const float* comp, const int32_t* n, const float* pos,
                              const float* prev, int batch, float track_len, float dt,
                              uint16_t* x, int32_t* slot_comp, const double* probs,
                              float* target, void* stream) {
    if (!comp || !n || !pos || !prev || !x) return fail(BBE_EINVAL, "NULL argument");
    if ((probs == nullptr) != (target == nullptr))
        return fail(BBE_EINVAL, "probs and target go together");
    if (batch < 1) return fail(BBE_EINVAL, "batch must be >= 1");
    if (reinterpret_cast<uintptr_t>(x) & 15u)
        return fail(BBE_EINVAL, "x must be 16-byte aligned");
    if (!std::isfinite(track_len) || !(track_len > 0.0f) || !std::isfinite(dt) || !(dt > 0.0f))
        return fail(BBE_EINVAL, "track_len and dt must be finite and > 0");
    bbe::EncodeArgs a;
    a.comp = comp;
    a.n = n;
    a.pos = pos;
    a.prev = prev;
    a.B = batch;
    a.track_len = track_len;
    a.c75 = 7.5f * dt;
    a.c15 = 15.0f * dt;
    a.c750 = 75.0f * dt;
    a.x = x;
    a.slot = slot_comp;
    a.probs_in = probs;
    a.target = target;
    hipError_t e = BBE_HIP(bbe::launch_encode(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching the encoder");
    return ok();
}
