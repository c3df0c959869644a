// The U-Net surrogate: parameters, forward, backward, Adam and tile
// inference, all as launches of the layer kernels in k_nn.hip.
//
// Network (encoder 16/32/64/128 channels, three 2x2 max pools, decoder with
// 2x2 stride-2 up-convolutions and skip concatenation, 1x1 head to two logit
// maps: foreground and seeds).  Activations are bfloat16, accumulation and
// gradients of activations float32, parameters float32 masters with bfloat16
// operand copies repacked after every update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rtseg_unet.h"
#include "nn_internal.h"
#include "rt_internal.h"

using namespace rtseg;

namespace {

enum Kind { CONV3 = 0, UP2 = 1, HEAD = 2 };

struct Layer {
    const char *name;
    Kind kind;
    int ci, co;         // ci is the padded input channel count for conv3 (multiple of 8)
    int64_t w_off, b_off, nw;
    bf16_t *wf = nullptr, *wt = nullptr;   // operand copies (conv3: [co][9][ci], [ci][9][co]; up2: [4][co][ci], [ci][4][co])
};

constexpr int CH[4] = {16, 32, 64, 128};
constexpr int IN_PAD = 8;
constexpr int WIN = 512;       // inference window
constexpr int WIN_STRIDE = 480;

std::vector<Layer> make_layers() {
    std::vector<Layer> L;
    auto conv = [&](const char *n, int ci, int co) { L.push_back(Layer{n, CONV3, ci, co, 0, 0, 0}); };
    auto up = [&](const char *n, int ci, int co) { L.push_back(Layer{n, UP2, ci, co, 0, 0, 0}); };
    conv("e1a", IN_PAD, CH[0]);
    conv("e1b", CH[0], CH[0]);
    conv("e2a", CH[0], CH[1]);
    conv("e2b", CH[1], CH[1]);
    conv("e3a", CH[1], CH[2]);
    conv("e3b", CH[2], CH[2]);
    conv("e4a", CH[2], CH[3]);
    conv("e4b", CH[3], CH[3]);
    up("u3", CH[3], CH[2]);
    conv("d3a", 2 * CH[2], CH[2]);
    conv("d3b", CH[2], CH[2]);
    up("u2", CH[2], CH[1]);
    conv("d2a", 2 * CH[1], CH[1]);
    conv("d2b", CH[1], CH[1]);
    up("u1", CH[1], CH[0]);
    conv("d1a", 2 * CH[0], CH[0]);
    conv("d1b", CH[0], CH[0]);
    L.push_back(Layer{"head", HEAD, CH[0], 2, 0, 0, 0});
    int64_t off = 0;
    for (Layer &l : L) {
        l.nw = l.kind == CONV3 ? (int64_t)l.co * 9 * l.ci : l.kind == UP2 ? (int64_t)l.ci * 4 * l.co : 2 * 16;
        l.w_off = off;
        off += l.nw;
        l.b_off = off;
        off += l.co;
    }
    return L;
}

int64_t total_params() {
    int64_t n = 0;
    for (const Layer &l : make_layers()) n += l.nw + l.co;
    return n;
}

// counter-based normal variates: splitmix64 of (seed, index), Box-Muller
uint64_t splitmix(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
double normal_at(uint64_t seed, uint64_t i) {
    const double u1 = ((splitmix(seed * 0x100000001b3ull + 2 * i) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix(seed * 0x100000001b3ull + 2 * i + 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// device buffer helper
template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return RT_OK;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("unet: allocation of %zu bytes failed", count * sizeof(T));
        return RT_ENOMEM;
    }
    return RT_OK;
}

}  // namespace

// Activations and gradient buffers of one batch shape (n, h, w).
struct Acts {
    int n = 0, h = 0, w = 0;
    bool train = false;
    std::vector<void *> bufs;
    bf16_t *x0 = nullptr;
    bf16_t *e[4][2] = {};        // encoder outputs (a, b) per level
    bf16_t *pool[3] = {};        // pooled skips
    uint8_t *idx[3] = {};
    bf16_t *u[3] = {};           // up-convolution outputs, level 0..2
    bf16_t *d[3][2] = {};        // decoder outputs (a, b) per level
    float *F1 = nullptr, *F2 = nullptr, *dS[3] = {};
    bf16_t *G = nullptr;
    int32_t *origin = nullptr;   // ox[n], oy[n], keep[4n]
};

struct rt_unet {
    int device = 0;
    std::vector<Layer> layers;
    int64_t np = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    bf16_t *packed = nullptr;
    int step = 0;
    Acts acts;
    // window origins of a whole tile inference (device, pinned host copy, the
    // event after its upload): uploaded once per call, so the window chunks
    // run back to back with no host wait
    int32_t *win_dev = nullptr, *win_host = nullptr;
    int64_t win_cap = 0;
    hipEvent_t win_done = nullptr;
    bool win_pending = false;
};

namespace {

void free_acts(Acts &a) {
    for (void *p : a.bufs) (void)hipFree(p);
    a = Acts{};
}

int ensure_acts(rt_unet *net, int n, int h, int w, bool train) {
    Acts &a = net->acts;
    if (a.n == n && a.h == h && a.w == w && (a.train || !train) && a.x0) return RT_OK;
    (void)hipDeviceSynchronize();
    free_acts(a);
    a.n = n;
    a.h = h;
    a.w = w;
    a.train = train;
    int e = RT_OK;
    auto bf = [&](bf16_t **p, int64_t count) {
        if (!e) e = dalloc(p, (size_t)count);
        if (!e) a.bufs.push_back(*p);
    };
    auto f32 = [&](float **p, int64_t count) {
        if (!e) e = dalloc(p, (size_t)count);
        if (!e) a.bufs.push_back(*p);
    };
    int64_t Pl[4];
    for (int l = 0; l < 4; ++l) Pl[l] = (int64_t)n * (h >> l) * (w >> l);
    bf(&a.x0, Pl[0] * IN_PAD);
    for (int l = 0; l < 4; ++l) {
        bf(&a.e[l][0], Pl[l] * CH[l]);
        bf(&a.e[l][1], Pl[l] * CH[l]);
    }
    for (int l = 0; l < 3; ++l) {
        bf(&a.pool[l], Pl[l + 1] * CH[l]);
        if (!e) e = dalloc(&a.idx[l], (size_t)(Pl[l + 1] * CH[l]));
        if (!e) a.bufs.push_back(a.idx[l]);
        bf(&a.u[l], Pl[l] * CH[l]);
        bf(&a.d[l][0], Pl[l] * CH[l]);
        bf(&a.d[l][1], Pl[l] * CH[l]);
    }
    if (train) {
        f32(&a.F1, Pl[0] * CH[0]);
        f32(&a.F2, Pl[0] * CH[0]);
        for (int l = 0; l < 3; ++l) f32(&a.dS[l], Pl[l] * CH[l]);
        bf(&a.G, Pl[0] * CH[0]);
    }
    if (!e) e = dalloc(&a.origin, (size_t)6 * n);
    if (!e) a.bufs.push_back(a.origin);
    if (e) free_acts(a);
    return e;
}

const Layer &layer(rt_unet *net, const char *name) {
    for (const Layer &l : net->layers)
        if (!std::strcmp(l.name, name)) return l;
    return net->layers[0];
}

int pack_all(rt_unet *net, hipStream_t s) {
    for (Layer &l : net->layers) {
        int e = RT_OK;
        if (l.kind == CONV3) e = nn_pack_conv3(net->P + l.w_off, l.co, l.ci, l.wf, l.wt, s);
        if (l.kind == UP2) e = nn_pack_up2(net->P + l.w_off, l.ci, l.co, l.wf, l.wt, s);
        if (e) return e;
    }
    return RT_OK;
}

// forward through the whole network on net->acts (input already in x0)
int forward(rt_unet *net, hipStream_t s) {
    Acts &a = net->acts;
    const int n = a.n;
    auto W = [&](const char *nm) -> const Layer & { return layer(net, nm); };
    int e;
    const bf16_t *in = a.x0;
    int cin = IN_PAD;
    static const char *enc[4][2] = {{"e1a", "e1b"}, {"e2a", "e2b"}, {"e3a", "e3b"}, {"e4a", "e4b"}};
    for (int l = 0; l < 4; ++l) {
        const int h = a.h >> l, w = a.w >> l;
        const Layer &A = W(enc[l][0]), &B = W(enc[l][1]);
        if ((e = nn_conv3_fwd(in, cin, nullptr, 0, n, h, w, A.wf, net->P + A.b_off, A.co, 1, a.e[l][0], nullptr, s)))
            return e;
        if ((e = nn_conv3_fwd(a.e[l][0], A.co, nullptr, 0, n, h, w, B.wf, net->P + B.b_off, B.co, 1, a.e[l][1],
                              nullptr, s)))
            return e;
        if (l < 3) {
            if ((e = nn_pool2_fwd(a.e[l][1], CH[l], n, h, w, a.pool[l], a.idx[l], s))) return e;
            in = a.pool[l];
            cin = CH[l];
        }
    }
    static const char *dec[3][3] = {{"u1", "d1a", "d1b"}, {"u2", "d2a", "d2b"}, {"u3", "d3a", "d3b"}};
    const bf16_t *below = a.e[3][1];
    for (int l = 2; l >= 0; --l) {
        const int h = a.h >> l, w = a.w >> l;
        const Layer &U = W(dec[l][0]), &A = W(dec[l][1]), &B = W(dec[l][2]);
        if ((e = nn_up2_fwd(below, U.ci, n, h / 2, w / 2, U.wf, net->P + U.b_off, U.co, a.u[l], nullptr, s))) return e;
        if ((e = nn_conv3_fwd(a.u[l], CH[l], a.e[l][1], CH[l], n, h, w, A.wf, net->P + A.b_off, A.co, 1, a.d[l][0],
                              nullptr, s)))
            return e;
        if ((e = nn_conv3_fwd(a.d[l][0], A.co, nullptr, 0, n, h, w, B.wf, net->P + B.b_off, B.co, 1, a.d[l][1],
                              nullptr, s)))
            return e;
        below = a.d[l][1];
    }
    return RT_OK;
}

// gradient of one conv3 layer: dy (f32, post-activation) -> G; dw, db; dx
int conv3_back(rt_unet *net, const Layer &L, const float *dy, const bf16_t *yout, const bf16_t *x0, int c0,
               const bf16_t *x1, int c1, int n, int h, int w, float *dx0, float *dx1, int split, hipStream_t s) {
    Acts &a = net->acts;
    const int64_t P = (int64_t)n * h * w;
    int e;
    if ((e = nn_relu_bwd(dy, yout, P * L.co, a.G, s))) return e;
    if ((e = nn_conv3_wgrad(x0, c0, x1, c1, a.G, L.co, n, h, w, net->G + L.w_off, s))) return e;
    if ((e = nn_colsum(a.G, L.co, P, net->G + L.b_off, s))) return e;
    if (dx0) return nn_conv3_dgrad(a.G, L.co, n, h, w, L.wt, L.ci, split, dx0, dx1, s);
    return RT_OK;
}

int backward(rt_unet *net, const uint8_t *t_fg, const uint8_t *t_seed, float w_seed, float *loss, hipStream_t s) {
    Acts &a = net->acts;
    const int n = a.n;
    auto W = [&](const char *nm) -> const Layer & { return layer(net, nm); };
    int e;
    const Layer &H = W("head");
    HeadArgs ha{};
    ha.x = a.d[0][1];
    ha.n = n;
    ha.h = a.h;
    ha.w = a.w;
    ha.wh = net->P + H.w_off;
    ha.bh = net->P + H.b_off;
    ha.t_fg = t_fg;
    ha.t_seed = t_seed;
    ha.w_seed = w_seed;
    ha.loss = loss;
    ha.dx = a.F1;
    ha.dw = net->G + H.w_off;
    ha.db = net->G + H.b_off;
    if ((e = nn_head(ha, s))) return e;
    static const char *dec[3][3] = {{"u1", "d1a", "d1b"}, {"u2", "d2a", "d2b"}, {"u3", "d3a", "d3b"}};
    // decoder, level 0 up to level 2; F1 holds the gradient of the level's output
    for (int l = 0; l < 3; ++l) {
        const int h = a.h >> l, w = a.w >> l;
        const Layer &U = W(dec[l][0]), &A = W(dec[l][1]), &B = W(dec[l][2]);
        if ((e = conv3_back(net, B, a.F1, a.d[l][1], a.d[l][0], CH[l], nullptr, 0, n, h, w, a.F2, nullptr, B.ci, s)))
            return e;
        if ((e = conv3_back(net, A, a.F2, a.d[l][0], a.u[l], CH[l], a.e[l][1], CH[l], n, h, w, a.F1, a.dS[l], CH[l],
                            s)))
            return e;
        // up-convolution: no activation after it
        const int64_t Pl = (int64_t)n * h * w;
        if ((e = nn_relu_bwd(a.F1, nullptr, Pl * U.co, a.G, s))) return e;
        const bf16_t *uin = l < 2 ? a.d[l + 1][1] : a.e[3][1];
        if ((e = nn_up2_wgrad(uin, U.ci, a.G, U.co, n, h / 2, w / 2, net->G + U.w_off, s))) return e;
        if ((e = nn_colsum(a.G, U.co, Pl, net->G + U.b_off, s))) return e;
        if ((e = nn_up2_dgrad(a.G, U.co, n, h / 2, w / 2, U.wt, U.ci, a.F1, s))) return e;
    }
    // encoder, level 3 down to level 0; F1 holds the gradient of e[l][1]
    static const char *enc[4][2] = {{"e1a", "e1b"}, {"e2a", "e2b"}, {"e3a", "e3b"}, {"e4a", "e4b"}};
    for (int l = 3; l >= 0; --l) {
        const int h = a.h >> l, w = a.w >> l;
        const Layer &A = W(enc[l][0]), &B = W(enc[l][1]);
        const float *dyb = a.F1;
        if (l < 3) {
            // the skip gradient plus the un-pooled gradient from below
            if ((e = nn_pool2_bwd(a.F1, a.idx[l], CH[l], n, h, w, a.dS[l], s))) return e;
            dyb = a.dS[l];
        }
        if ((e = conv3_back(net, B, dyb, a.e[l][1], a.e[l][0], CH[l], nullptr, 0, n, h, w, a.F2, nullptr, B.ci, s)))
            return e;
        const bf16_t *xin = l > 0 ? a.pool[l - 1] : a.x0;
        const int cin = l > 0 ? CH[l - 1] : IN_PAD;
        if ((e = conv3_back(net, A, a.F2, a.e[l][0], xin, cin, nullptr, 0, n, h, w, l > 0 ? a.F1 : nullptr, nullptr,
                            A.ci, s)))
            return e;
    }
    return RT_OK;
}

}  // namespace

extern "C" {

int64_t rt_unet_param_count(void) { return total_params(); }

int rt_unet_create(rt_ctx *ctx, uint64_t seed, rt_unet **out) {
    if (!out) {
        set_error("rt_unet_create: out is NULL");
        return RT_EINVAL;
    }
    *out = nullptr;
    int dev = 0;
    if (ctx) {
        int e = rt_get_knob(ctx, "device", &dev);
        if (e) dev = 0;
    }
    RT_HIP(hipSetDevice(dev));
    rt_unet *net = new rt_unet();
    net->device = dev;
    net->layers = make_layers();
    net->np = total_params();
    int64_t npk = 0;
    for (const Layer &l : net->layers)
        if (l.kind != HEAD) npk += 2 * l.nw;
    int e = dalloc(&net->P, net->np);
    if (!e) e = dalloc(&net->G, net->np);
    if (!e) e = dalloc(&net->M, net->np);
    if (!e) e = dalloc(&net->V, net->np);
    if (!e) e = dalloc(&net->packed, npk);
    if (e) {
        rt_unet_destroy(net);
        return e;
    }
    bf16_t *q = net->packed;
    for (Layer &l : net->layers) {
        if (l.kind == HEAD) continue;
        l.wf = q;
        q += l.nw;
        l.wt = q;
        q += l.nw;
    }
    // He-normal weights (fan-in of the true input channels), zero biases and
    // zero weights on the padded input channels of the first layer
    std::vector<float> h(net->np, 0.f);
    uint64_t tensor = 0;
    for (const Layer &l : net->layers) {
        ++tensor;
        const int true_ci = !std::strcmp(l.name, "e1a") ? 3 : l.ci;
        const double fan = l.kind == CONV3 ? 9.0 * true_ci : l.kind == UP2 ? (double)l.ci : 16.0;
        const double sd = std::sqrt(2.0 / fan);
        for (int64_t i = 0; i < l.nw; ++i) {
            if (l.kind == CONV3 && (int)(i % l.ci) >= true_ci) continue;
            h[l.w_off + i] = (float)(sd * normal_at(seed ^ (tensor << 48), (uint64_t)i));
        }
    }
    if (hipMemcpy(net->P, h.data(), sizeof(float) * net->np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->G, 0, sizeof(float) * net->np) != hipSuccess ||
        hipMemset(net->M, 0, sizeof(float) * net->np) != hipSuccess ||
        hipMemset(net->V, 0, sizeof(float) * net->np) != hipSuccess) {
        (void)hipGetLastError();
        rt_unet_destroy(net);
        set_error("rt_unet_create: initialisation copy failed");
        return RT_EDEVICE;
    }
    if ((e = pack_all(net, nullptr)) || (e = hip_fail(hipDeviceSynchronize(), "rt_unet_create"))) {
        rt_unet_destroy(net);
        return e;
    }
    *out = net;
    return RT_OK;
}

int rt_unet_destroy(rt_unet *net) {
    if (!net) return RT_OK;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    free_acts(net->acts);
    for (void *p : {(void *)net->P, (void *)net->G, (void *)net->M, (void *)net->V, (void *)net->packed})
        if (p) (void)hipFree(p);
    if (net->win_dev) (void)hipFree(net->win_dev);
    if (net->win_host) (void)hipHostFree(net->win_host);
    if (net->win_done) (void)hipEventDestroy(net->win_done);
    delete net;
    return RT_OK;
}

int rt_unet_get_params(rt_unet *net, float *host, int64_t count) {
    if (!net || !host || count != net->np) {
        set_error("rt_unet_get_params: bad arguments (count must be %lld)", (long long)(net ? net->np : 0));
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    RT_HIP(hipDeviceSynchronize());
    RT_HIP(hipMemcpy(host, net->P, sizeof(float) * count, hipMemcpyDeviceToHost));
    return RT_OK;
}

int rt_unet_set_params(rt_unet *net, const float *host, int64_t count) {
    if (!net || !host || count != net->np) {
        set_error("rt_unet_set_params: bad arguments (count must be %lld)", (long long)(net ? net->np : 0));
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    RT_HIP(hipDeviceSynchronize());
    RT_HIP(hipMemcpy(net->P, host, sizeof(float) * count, hipMemcpyHostToDevice));
    RT_HIP(hipMemset(net->M, 0, sizeof(float) * count));
    RT_HIP(hipMemset(net->V, 0, sizeof(float) * count));
    RT_HIP(hipMemset(net->G, 0, sizeof(float) * count));
    net->step = 0;
    int e = pack_all(net, nullptr);
    if (e) return e;
    RT_HIP(hipDeviceSynchronize());
    return RT_OK;
}

int rt_unet_get_grads(rt_unet *net, float *host, int64_t count) {
    if (!net || !host || count != net->np) {
        set_error("rt_unet_get_grads: bad arguments");
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    RT_HIP(hipDeviceSynchronize());
    RT_HIP(hipMemcpy(host, net->G, sizeof(float) * count, hipMemcpyDeviceToHost));
    return RT_OK;
}

int rt_unet_grad_step(rt_unet *net, const uint8_t *rgb, const uint8_t *fg_tgt, const uint8_t *seed_tgt, int32_t b,
                      int32_t h, int32_t w, float w_seed, float *loss_dev, void *stream) {
    if (!net || !rgb || !fg_tgt || !seed_tgt || !loss_dev || b <= 0 || h <= 0 || w <= 0 || h % 8 || w % 8) {
        set_error("rt_unet_grad_step: bad arguments (h and w must be positive multiples of 8)");
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    hipStream_t s = (hipStream_t)stream;
    int e = ensure_acts(net, b, h, w, true);
    if (e) return e;
    // the batch is one tall image: window k starts at row k*h
    std::vector<int32_t> org(6 * (size_t)b, 0);
    for (int k = 0; k < b; ++k) org[b + k] = k * h;
    RT_HIP(hipMemcpyAsync(net->acts.origin, org.data(), sizeof(int32_t) * 2 * b, hipMemcpyHostToDevice, s));
    if ((e = nn_prep_input(rgb, 3LL * w, w, b * h, net->acts.origin, net->acts.origin + b, b, h, w, net->acts.x0, s)))
        return e;
    if ((e = nn_fill_f32(loss_dev, 0.f, 1, s))) return e;
    if ((e = forward(net, s))) return e;
    if ((e = backward(net, fg_tgt, seed_tgt, w_seed, loss_dev, s))) return e;
    // the host copy of the origins must outlive the asynchronous copy
    RT_HIP(hipStreamSynchronize(s));
    return RT_OK;
}

int rt_unet_adam_step(rt_unet *net, float lr, void *stream) {
    if (!net || !std::isfinite(lr)) {
        set_error("rt_unet_adam_step: bad arguments");
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    hipStream_t s = (hipStream_t)stream;
    net->step++;
    int e = nn_adam(net->P, net->G, net->M, net->V, net->np, lr, 0.9f, 0.999f, 1e-8f, net->step, s);
    if (e) return e;
    return pack_all(net, s);
}

int rt_unet_train_step(rt_unet *net, const uint8_t *rgb, const uint8_t *fg_tgt, const uint8_t *seed_tgt, int32_t b,
                       int32_t h, int32_t w, float lr, float w_seed, float *loss_dev, void *stream) {
    int e = rt_unet_grad_step(net, rgb, fg_tgt, seed_tgt, b, h, w, w_seed, loss_dev, stream);
    if (e) return e;
    return rt_unet_adam_step(net, lr, stream);
}

int rt_unet_get_step(rt_unet *net, int64_t *step) {
    if (!net || !step) {
        set_error("rt_unet_get_step: null argument");
        return RT_EINVAL;
    }
    *step = net->step;
    return RT_OK;
}

int rt_unet_forward(rt_unet *net, const uint8_t *rgb, int64_t rgb_pitch, int32_t w, int32_t h, float *fg_prob,
                    float *seed_prob, int64_t prob_pitch, void *stream) {
    if (!net || !rgb || !fg_prob || !seed_prob || w <= 0 || h <= 0 || rgb_pitch < 3LL * w || prob_pitch < w) {
        set_error("rt_unet_forward: bad arguments");
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    hipStream_t s = (hipStream_t)stream;
    // window origins: stride 480, the last window flush with the tile edge;
    // each window keeps the part of its overlaps nearer to its own centre
    // along an axis shorter than a window the window shrinks to the axis
    // length rounded up to a multiple of 8 (zero input beyond the tile)
    auto axis = [](int len, int &win, std::vector<int> &pos, std::vector<int> &lo, std::vector<int> &hi) {
        pos.clear();
        win = std::min(WIN, (len + 7) / 8 * 8);
        if (len <= win) {
            pos.push_back(0);
        } else {
            for (int p = 0;; p += WIN_STRIDE) {
                if (p + win >= len) {
                    pos.push_back(len - win);
                    break;
                }
                pos.push_back(p);
            }
        }
        const int k = (int)pos.size();
        lo.assign(k, 0);
        hi.assign(k, win);
        for (int i = 0; i < k; ++i) {
            if (i > 0) lo[i] = (pos[i - 1] + win + pos[i]) / 2 - pos[i];
            if (i + 1 < k) hi[i] = (pos[i] + win + pos[i + 1]) / 2 - pos[i];
        }
    };
    std::vector<int> px, pxl, pxh, py, pyl, pyh;
    int win_w = WIN, win_h = WIN;
    axis(w, win_w, px, pxl, pxh);
    axis(h, win_h, py, pyl, pyh);
    const int nwin = (int)(px.size() * py.size());
    const int chunk = std::min(nwin, 16);
    int e = ensure_acts(net, chunk, win_h, win_w, false);
    if (e) return e;
    const Layer &H = layer(net, "head");
    // every chunk's origins (ox[nb], oy[nb], keep[4 nb]) back to back, one upload
    const int64_t need = 6 * (int64_t)nwin;
    if (net->win_pending) {   // the previous call's upload may still read the host copy
        RT_HIP(hipEventSynchronize(net->win_done));
        net->win_pending = false;
    }
    if (need > net->win_cap) {
        RT_HIP(hipDeviceSynchronize());
        if (net->win_dev) RT_HIP(hipFree(net->win_dev));
        if (net->win_host) RT_HIP(hipHostFree(net->win_host));
        net->win_dev = net->win_host = nullptr;
        net->win_cap = 0;
        if (hipMalloc((void **)&net->win_dev, sizeof(int32_t) * need) != hipSuccess ||
            hipHostMalloc((void **)&net->win_host, sizeof(int32_t) * need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("rt_unet_forward: window origin buffers");
            return RT_ENOMEM;
        }
        net->win_cap = need;
    }
    if (!net->win_done) RT_HIP(hipEventCreateWithFlags(&net->win_done, hipEventDisableTiming));
    for (int c0 = 0; c0 < nwin; c0 += chunk) {
        const int nb = std::min(chunk, nwin - c0);
        int32_t *org = net->win_host + 6 * (int64_t)c0;
        for (int k = 0; k < nb; ++k) {
            const int wi = c0 + k;
            const int ix = wi % (int)px.size(), iy = wi / (int)px.size();
            org[k] = px[ix];
            org[nb + k] = py[iy];
            org[2 * nb + 4 * k + 0] = pxl[ix];
            org[2 * nb + 4 * k + 1] = pxh[ix];
            org[2 * nb + 4 * k + 2] = pyl[iy];
            org[2 * nb + 4 * k + 3] = pyh[iy];
        }
    }
    RT_HIP(hipMemcpyAsync(net->win_dev, net->win_host, sizeof(int32_t) * need, hipMemcpyHostToDevice, s));
    RT_HIP(hipEventRecord(net->win_done, s));
    net->win_pending = true;
    for (int c0 = 0; c0 < nwin; c0 += chunk) {
        const int nb = std::min(chunk, nwin - c0);
        int32_t *dorg = net->win_dev + 6 * (int64_t)c0;
        net->acts.n = nb;
        if ((e = nn_prep_input(rgb, rgb_pitch, w, h, dorg, dorg + nb, nb, win_h, win_w, net->acts.x0, s))) return e;
        if ((e = forward(net, s))) return e;
        HeadArgs ha{};
        ha.x = net->acts.d[0][1];
        ha.n = nb;
        ha.h = win_h;
        ha.w = win_w;
        ha.wh = net->P + H.w_off;
        ha.bh = net->P + H.b_off;
        ha.p_fg = fg_prob;
        ha.p_seed = seed_prob;
        ha.pitch = prob_pitch;
        ha.ox = dorg;
        ha.oy = dorg + nb;
        ha.keep = dorg + 2 * nb;
        ha.out_w = w;
        ha.out_h = h;
        if ((e = nn_head(ha, s))) return e;
    }
    net->acts.n = chunk;
    return RT_OK;
}

int rt_unet_save(rt_unet *net, const char *path) {
    if (!net || !path) {
        set_error("rt_unet_save: null argument");
        return RT_EINVAL;
    }
    std::vector<float> h(net->np);
    int e = rt_unet_get_params(net, h.data(), net->np);
    if (e) return e;
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("rt_unet_save: cannot open %s", path);
        return RT_EINVAL;
    }
    const char magic[8] = {'R', 'T', 'U', 'N', 'E', 'T', '0', '1'};
    const int64_t n = net->np;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, sizeof n, 1, f) == 1 &&
              std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_error("rt_unet_save: write to %s failed", path);
        return RT_EDEVICE;
    }
    return RT_OK;
}

int rt_unet_load(rt_unet *net, const char *path) {
    if (!net || !path) {
        set_error("rt_unet_load: null argument");
        return RT_EINVAL;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("rt_unet_load: cannot open %s", path);
        return RT_EINVAL;
    }
    char magic[8];
    int64_t n = 0;
    std::vector<float> h(net->np);
    bool ok = std::fread(magic, 1, 8, f) == 8 && !std::memcmp(magic, "RTUNET01", 8) &&
              std::fread(&n, sizeof n, 1, f) == 1 && n == net->np &&
              std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) {
        set_error("rt_unet_load: %s is not a parameter file of this network", path);
        return RT_EINVAL;
    }
    return rt_unet_set_params(net, h.data(), net->np);
}

// Training checkpoint: 8 magic bytes "RTUNETC1", int64 count, int64 step,
// then count float32 each of the master weights, the gradient accumulator and
// the two Adam moments.
int rt_unet_save_checkpoint(rt_unet *net, const char *path) {
    if (!net || !path) {
        set_error("rt_unet_save_checkpoint: null argument");
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    RT_HIP(hipDeviceSynchronize());
    const int64_t n = net->np, step = net->step;
    std::vector<float> h((size_t)n * 4);
    const float *src[4] = {net->P, net->G, net->M, net->V};
    for (int k = 0; k < 4; ++k)
        RT_HIP(hipMemcpy(h.data() + (size_t)k * n, src[k], sizeof(float) * n, hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("rt_unet_save_checkpoint: cannot open %s", path);
        return RT_EINVAL;
    }
    const char magic[8] = {'R', 'T', 'U', 'N', 'E', 'T', 'C', '1'};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, sizeof n, 1, f) == 1 &&
              std::fwrite(&step, sizeof step, 1, f) == 1 && std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_error("rt_unet_save_checkpoint: write to %s failed", path);
        return RT_EDEVICE;
    }
    return RT_OK;
}

int rt_unet_load_checkpoint(rt_unet *net, const char *path) {
    if (!net || !path) {
        set_error("rt_unet_load_checkpoint: null argument");
        return RT_EINVAL;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("rt_unet_load_checkpoint: cannot open %s", path);
        return RT_EINVAL;
    }
    char magic[8];
    int64_t n = 0, step = 0;
    std::vector<float> h((size_t)net->np * 4);
    bool ok = std::fread(magic, 1, 8, f) == 8 && !std::memcmp(magic, "RTUNETC1", 8) &&
              std::fread(&n, sizeof n, 1, f) == 1 && n == net->np && std::fread(&step, sizeof step, 1, f) == 1 &&
              step >= 0 && std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) {
        set_error("rt_unet_load_checkpoint: %s is not a checkpoint of this network", path);
        return RT_EINVAL;
    }
    RT_HIP(hipSetDevice(net->device));
    RT_HIP(hipDeviceSynchronize());
    float *dst[4] = {net->P, net->G, net->M, net->V};
    for (int k = 0; k < 4; ++k)
        RT_HIP(hipMemcpy(dst[k], h.data() + (size_t)k * n, sizeof(float) * n, hipMemcpyHostToDevice));
    net->step = (int)step;
    int e = pack_all(net, nullptr);
    if (e) return e;
    RT_HIP(hipDeviceSynchronize());
    return RT_OK;
}

// ---------------------------------------------------------------------------
// single layers through the C ABI (bfloat16 operands, float32 results)
// ---------------------------------------------------------------------------

int rt_nn_conv3_fwd(rt_ctx *ctx, const uint16_t *x0, int32_t c0, const uint16_t *x1, int32_t c1, int32_t n,
                    int32_t h, int32_t w, const uint16_t *wf, const float *bias, int32_t co, int32_t relu, float *y_f32,
                    uint16_t *y_bf16, void *stream) {
    (void)ctx;
    if (!x0 || !wf || !bias || (!y_f32 && !y_bf16) || n <= 0 || h <= 0 || w <= 0) {
        set_error("rt_nn_conv3_fwd: bad arguments");
        return RT_EINVAL;
    }
    return nn_conv3_fwd(x0, c0, x1, c1, n, h, w, wf, bias, co, relu, y_bf16, y_f32, (hipStream_t)stream);
}

int rt_nn_conv3_dgrad(rt_ctx *ctx, const uint16_t *g, int32_t co, int32_t n, int32_t h, int32_t w, const uint16_t *wt,
                      int32_t ci, int32_t c0, float *dx0, float *dx1, void *stream) {
    (void)ctx;
    if (!g || !wt || !dx0 || n <= 0 || h <= 0 || w <= 0) {
        set_error("rt_nn_conv3_dgrad: bad arguments");
        return RT_EINVAL;
    }
    return nn_conv3_dgrad(g, co, n, h, w, wt, ci, c0, dx0, dx1, (hipStream_t)stream);
}

int rt_nn_conv3_wgrad(rt_ctx *ctx, const uint16_t *x0, int32_t c0, const uint16_t *x1, int32_t c1, const uint16_t *g,
                      int32_t co, int32_t n, int32_t h, int32_t w, float *dw, float *db, void *stream) {
    (void)ctx;
    if (!x0 || !g || !dw || n <= 0 || h <= 0 || w <= 0) {
        set_error("rt_nn_conv3_wgrad: bad arguments");
        return RT_EINVAL;
    }
    int e = nn_conv3_wgrad(x0, c0, x1, c1, g, co, n, h, w, dw, (hipStream_t)stream);
    if (!e && db) e = nn_colsum(g, co, (int64_t)n * h * w, db, (hipStream_t)stream);
    return e;
}

int rt_nn_up2_fwd(rt_ctx *ctx, const uint16_t *x, int32_t ci, int32_t n, int32_t h, int32_t w, const uint16_t *uf,
                  const float *bias, int32_t co, float *y_f32, uint16_t *y_bf16, void *stream) {
    (void)ctx;
    if (!x || !uf || !bias || (!y_f32 && !y_bf16) || n <= 0 || h <= 0 || w <= 0) {
        set_error("rt_nn_up2_fwd: bad arguments");
        return RT_EINVAL;
    }
    return nn_up2_fwd(x, ci, n, h, w, uf, bias, co, y_bf16, y_f32, (hipStream_t)stream);
}

int rt_nn_up2_bwd(rt_ctx *ctx, const uint16_t *x, int32_t ci, const uint16_t *g, int32_t co, int32_t n, int32_t h,
                  int32_t w, const uint16_t *ut, float *dx, float *dw, float *db, void *stream) {
    (void)ctx;
    if (!x || !g || !ut || n <= 0 || h <= 0 || w <= 0) {
        set_error("rt_nn_up2_bwd: bad arguments");
        return RT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int e = RT_OK;
    if (dx) e = nn_up2_dgrad(g, co, n, h, w, ut, ci, dx, s);
    if (!e && dw) e = nn_up2_wgrad(x, ci, g, co, n, h, w, dw, s);
    if (!e && db) e = nn_colsum(g, co, (int64_t)n * 4 * h * w, db, s);
    return e;
}

int rt_nn_pool2(rt_ctx *ctx, const uint16_t *x, int32_t c, int32_t n, int32_t h, int32_t w, uint16_t *y, uint8_t *idx,
                const float *dy, float *dx, void *stream) {
    (void)ctx;
    hipStream_t s = (hipStream_t)stream;
    if (x && y && idx) return nn_pool2_fwd(x, c, n, h, w, y, idx, s);
    if (dy && idx && dx) return nn_pool2_bwd(dy, idx, c, n, h, w, dx, s);
    set_error("rt_nn_pool2: give (x, y, idx) for the forward pass or (dy, idx, dx) for the backward pass");
    return RT_EINVAL;
}

int rt_nn_head_loss(rt_ctx *ctx, const uint16_t *x, int32_t n, int32_t h, int32_t w, const float *wh, const float *bh,
                    const uint8_t *t_fg, const uint8_t *t_seed, float w_seed, float *loss, float *dx, float *dw,
                    float *db, void *stream) {
    (void)ctx;
    if (!x || !wh || !bh || !t_fg || !t_seed || !loss || !dx || !dw || !db) {
        set_error("rt_nn_head_loss: null argument");
        return RT_EINVAL;
    }
    HeadArgs a{};
    a.x = x;
    a.n = n;
    a.h = h;
    a.w = w;
    a.wh = wh;
    a.bh = bh;
    a.t_fg = t_fg;
    a.t_seed = t_seed;
    a.w_seed = w_seed;
    a.loss = loss;
    a.dx = dx;
    a.dw = dw;
    a.db = db;
    return nn_head(a, (hipStream_t)stream);
}

int rt_nn_pack(rt_ctx *ctx, int32_t kind, const float *w, int32_t ci, int32_t co, uint16_t *fwd, uint16_t *tr,
               void *stream) {
    (void)ctx;
    if (!w || !fwd || !tr) {
        set_error("rt_nn_pack: null argument");
        return RT_EINVAL;
    }
    if (kind == 0) return nn_pack_conv3(w, co, ci, fwd, tr, (hipStream_t)stream);
    if (kind == 1) return nn_pack_up2(w, ci, co, fwd, tr, (hipStream_t)stream);
    set_error("rt_nn_pack: kind must be 0 (conv3) or 1 (up2)");
    return RT_EINVAL;
}

int rt_nn_prep_input(rt_ctx *ctx, const uint8_t *rgb, int64_t pitch, int32_t w, int32_t h, uint16_t *x, void *stream) {
    (void)ctx;
    if (!rgb || !x || w <= 0 || h <= 0) {
        set_error("rt_nn_prep_input: bad arguments");
        return RT_EINVAL;
    }
    // a single window at the origin covering the image
    static int32_t *zero = nullptr;
    if (!zero) {
        if (hipMalloc((void **)&zero, 2 * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            zero = nullptr;
            set_error("rt_nn_prep_input: allocation failed");
            return RT_ENOMEM;
        }
        RT_HIP(hipMemset(zero, 0, 2 * sizeof(int32_t)));
    }
    return nn_prep_input(rgb, pitch, w, h, zero, zero + 1, 1, h, w, x, (hipStream_t)stream);
}

}  // extern "C"
