// Host side of the proposal network: parameter layout, buffers, the forward
// and backward launch sequences, Adam, save/load (C-ABI in include/amhmvs.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "amh_ctx.h"
#include "amh_nn.h"

using namespace amh;
using namespace amh::nn;

namespace amh {

namespace {

// (c_in, c_out, kernel size) in canonical parameter order
struct LayerSpec {
    const char *name;
    int cin, cout, ks;
};
constexpr LayerSpec kSpec[] = {
    {"enc0a", 16, 16, 3}, {"enc0b", 16, 16, 3}, {"enc1a", 16, 32, 3}, {"enc1b", 32, 32, 3},
    {"enc2a", 32, 48, 3}, {"enc2b", 48, 48, 3}, {"enc3a", 48, 64, 3}, {"enc3b", 64, 64, 3},
    {"dec2", 112, 48, 3}, {"dec1", 80, 32, 3},  {"dec0", 48, 16, 3},  {"head", 16, 5, 1},
};
constexpr int kLayers = 12;
enum { ENC0A, ENC0B, ENC1A, ENC1B, ENC2A, ENC2B, ENC3A, ENC3B, DEC2, DEC1, DEC0, HEAD };
constexpr int kIn = 16;
constexpr char kMagic[8] = {'A', 'M', 'H', 'N', 'N', '0', '0', '1'};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Layer {
    int cin, cout, ks, cout_pad, kpad;
    size_t w_off, b_off;  // element offsets into the padded parameter arrays
};

int64_t canonical_count() {
    int64_t n = 0;
    for (const auto &l : kSpec) n += (int64_t)l.cout * l.ks * l.ks * l.cin + l.cout;
    return n;
}

}  // namespace

// buffers of one activation level
struct NetState {
    Layer L[kLayers];
    size_t n_pad = 0;                    // padded parameter count
    float *p32 = nullptr, *g32 = nullptr, *m = nullptr, *v = nullptr;
    bf16_t *pb = nullptr;                // bf16 copy of p32 (weights read from here)
    bf16_t *wt = nullptr;                // transposed weights of one layer
    size_t wt_cap = 0;
    float *part = nullptr, *bpart = nullptr;  // weight-gradient partial sums
    size_t part_cap = 0, bpart_cap = 0;
    float *loss_part = nullptr, *loss_dev = nullptr;
    size_t loss_cap = 0;
    int step = 0;
    // activations and gradients, sized for cap_px level-0 cells
    size_t cap_px = 0;
    std::vector<void *> bufs;
    float *qref;                         // depth base of the kept forward pass
    bf16_t *x, *e0a, *e0, *p0, *e1a, *e1, *p1, *e2a, *e2, *p2, *e3a, *e3, *c2, *d2, *c1, *d1, *c0, *d0;
    float *z;
    bf16_t *dz, *g_d0, *dc0, *g_d1, *dc1, *g_d2, *dc2, *g_e3, *g_e3a, *dp2, *g_e2, *g_e2a, *dp1, *g_e1, *g_e1a, *dp0,
        *g_e0, *g_e0a;
    int n = 0, h = 0, w = 0;
    bool have_fwd = false, have_grad = false;
};

void free_net(amh_ctx *c) {
    NetState *N = c->net;
    if (!N) return;
    for (void *p : {(void *)N->p32, (void *)N->g32, (void *)N->m, (void *)N->v, (void *)N->pb, (void *)N->wt,
                    (void *)N->part, (void *)N->bpart, (void *)N->loss_part, (void *)N->loss_dev})
        if (p) (void)hipFree(p);
    for (void *p : N->bufs)
        if (p) (void)hipFree(p);
    delete N;
    c->net = nullptr;
}

}  // namespace amh

namespace {

amh_status free_acts(NetState *N) {
    for (void *p : N->bufs)
        if (p) (void)hipFree(p);
    N->bufs.clear();
    N->cap_px = 0;
    return AMH_OK;
}

// (re)allocates activations and gradients for P0 level-0 cells
amh_status ensure_acts(amh_ctx *c, size_t P0) {
    NetState *N = c->net;
    if (P0 <= N->cap_px) return AMH_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_acts(N);
    const size_t P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
    amh_status st = AMH_OK;
    auto get = [&](size_t px, int ch) -> bf16_t * {
        void *p = nullptr;
        if (st == AMH_OK) st = dalloc(c, &p, px * ch * sizeof(bf16_t));
        N->bufs.push_back(p);
        return static_cast<bf16_t *>(p);
    };
    N->qref = reinterpret_cast<float *>(get(P0, 2));  // one float per cell
    N->x = get(P0, 16);
    N->e0a = get(P0, 16);
    N->e0 = get(P0, 16);
    N->p0 = get(P1, 16);
    N->e1a = get(P1, 32);
    N->e1 = get(P1, 32);
    N->p1 = get(P2, 32);
    N->e2a = get(P2, 48);
    N->e2 = get(P2, 48);
    N->p2 = get(P3, 48);
    N->e3a = get(P3, 64);
    N->e3 = get(P3, 64);
    N->c2 = get(P2, 112);
    N->d2 = get(P2, 48);
    N->c1 = get(P1, 80);
    N->d1 = get(P1, 32);
    N->c0 = get(P0, 48);
    N->d0 = get(P0, 16);
    N->z = reinterpret_cast<float *>(get(P0, 32));  // 16 floats per cell
    N->dz = get(P0, 16);
    N->g_d0 = get(P0, 16);
    N->dc0 = get(P0, 48);
    N->g_d1 = get(P1, 32);
    N->dc1 = get(P1, 80);
    N->g_d2 = get(P2, 48);
    N->dc2 = get(P2, 112);
    N->g_e3 = get(P3, 64);
    N->g_e3a = get(P3, 64);
    N->dp2 = get(P3, 48);
    N->g_e2 = get(P2, 48);
    N->g_e2a = get(P2, 48);
    N->dp1 = get(P2, 32);
    N->g_e1 = get(P1, 32);
    N->g_e1a = get(P1, 32);
    N->dp0 = get(P1, 16);
    N->g_e0 = get(P0, 16);
    N->g_e0a = get(P0, 16);
    if (st != AMH_OK) {
        free_acts(N);
        return st;
    }
    N->cap_px = P0;
    return AMH_OK;
}

// layer table, parameter buffers and the initial parameters (host vector in padded layout)
amh_status create_net(amh_ctx *c) {
    if (c->net) return AMH_OK;
    NetState *N = new (std::nothrow) NetState();
    if (!N) return fail(c, AMH_E_OOM, "host allocation failed");
    c->net = N;
    size_t off = 0;
    size_t wt_max = 0;
    for (int i = 0; i < kLayers; ++i) {
        Layer &l = N->L[i];
        l.cin = kSpec[i].cin;
        l.cout = kSpec[i].cout;
        l.ks = kSpec[i].ks;
        l.cout_pad = round_up(l.cout, 16);
        l.kpad = round_up(l.ks * l.ks * l.cin, 32);
        l.w_off = off;
        off += (size_t)l.cout_pad * l.kpad;
        l.b_off = off;
        off += (size_t)round_up(l.cout_pad, 64);
        wt_max = std::max(wt_max, (size_t)l.cin * round_up(l.ks * l.ks * l.cout_pad, 32));
    }
    N->n_pad = off;
    amh_status st = AMH_OK;
    if (st == AMH_OK) st = dalloc(c, (void **)&N->p32, off * 4);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->g32, off * 4);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->m, off * 4);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->v, off * 4);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->pb, off * 2);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->wt, wt_max * 2);
    if (st == AMH_OK) st = dalloc(c, (void **)&N->loss_dev, 64);
    if (st == AMH_OK && hipMemsetAsync(N->g32, 0, off * 4, c->stream) != hipSuccess)
        st = fail(c, AMH_E_HIP, "hipMemsetAsync of the gradient buffer failed");
    if (st != AMH_OK) {
        free_net(c);  // no half-built network stays on the context
        return st;
    }
    N->wt_cap = wt_max;
    return AMH_OK;
}

// canonical <-> padded parameter layout
void pack(const NetState *N, const float *canon, std::vector<float> &pad) {
    pad.assign(N->n_pad, 0.f);
    size_t o = 0;
    for (int i = 0; i < kLayers; ++i) {
        const Layer &l = N->L[i];
        const int K = l.ks * l.ks * l.cin;  // canonical weight [co][ky][kx][ci] is k = tap * cin + ci
        for (int co = 0; co < l.cout; ++co)
            for (int k = 0; k < K; ++k) pad[l.w_off + (size_t)co * l.kpad + k] = canon[o++];
        for (int co = 0; co < l.cout; ++co) pad[l.b_off + co] = canon[o++];
    }
}

void unpack(const NetState *N, const std::vector<float> &pad, float *canon) {
    size_t o = 0;
    for (int i = 0; i < kLayers; ++i) {
        const Layer &l = N->L[i];
        const int K = l.ks * l.ks * l.cin;
        for (int co = 0; co < l.cout; ++co)
            for (int k = 0; k < K; ++k) canon[o++] = pad[l.w_off + (size_t)co * l.kpad + k];
        for (int co = 0; co < l.cout; ++co) canon[o++] = pad[l.b_off + co];
    }
}

// uploads padded parameters, refreshes the bf16 copy, clears Adam
amh_status upload_params(amh_ctx *c, const std::vector<float> &pad) {
    NetState *N = c->net;
    HIPCHK(c, hipMemcpyAsync(N->p32, pad.data(), pad.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_to_bf16(N->p32, (int)N->n_pad, N->pb, c->stream));
    HIPCHK(c, hipMemsetAsync(N->m, 0, N->n_pad * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(N->v, 0, N->n_pad * 4, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // pad is the caller's host vector
    N->step = 0;
    N->have_fwd = false;
    N->have_grad = false;
    return AMH_OK;
}

// splitmix64 stream -> uniform (0, 1] -> standard normal (Box-Muller)
struct HostNormal {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((double)(next() >> 11) + 1.0) * 0x1p-53; }
    double normal() {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

ConvArgs conv_args(const Layer &l, const bf16_t *x, const bf16_t *w, const float *b, void *y, int n, int h, int wd,
                   int relu, int out_f32) {
    ConvArgs a;
    a.x = x;
    a.wgt = w;
    a.bias = b;
    a.mask = nullptr;
    a.y = y;
    a.n = n;
    a.h = h;
    a.w = wd;
    a.cin = l.cin;
    a.cout_pad = l.cout_pad;
    a.kpad = l.kpad;
    a.ks = l.ks;
    a.relu = relu;
    a.out_f32 = out_f32;
    return a;
}

amh_status conv_fwd(amh_ctx *c, int li, const bf16_t *x, void *y, int n, int h, int w, bool head, hipStream_t s) {
    NetState *N = c->net;
    const Layer &l = N->L[li];
    const ConvArgs a = conv_args(l, x, N->pb + l.w_off, N->p32 + l.b_off, y, n, h, w, head ? 0 : 1, head ? 1 : 0);
    HIPCHK(c, launch_conv(a, s));
    return AMH_OK;
}

// gradient of layer li with pre-activation gradient g (bf16 [P][cout_pad]) and input x:
// weight and bias gradients into g32; if dx != NULL the input gradient, masked by (mask > 0) if given
amh_status conv_bwd(amh_ctx *c, int li, const bf16_t *x, const bf16_t *g, bf16_t *dx, const bf16_t *mask, int n, int h,
                    int w) {
    NetState *N = c->net;
    const Layer &l = N->L[li];
    const int P = n * h * w;
    // weight gradient: splits of at least 256 cells, at most 64 splits
    int splits = std::max(1, std::min(64, (P + 255) / 256));
    int chunk = round_up((P + splits - 1) / splits, 32);
    splits = (P + chunk - 1) / chunk;
    const size_t need = (size_t)splits * l.cout_pad * l.kpad, needb = (size_t)splits * l.cout_pad;
    if (need > N->part_cap || needb > N->bpart_cap) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (N->part) (void)hipFree(N->part);
        if (N->bpart) (void)hipFree(N->bpart);
        N->part = N->bpart = nullptr;
        N->part_cap = N->bpart_cap = 0;
        const size_t cap = std::max(need, (size_t)64 * 48 * 1024), capb = std::max(needb, (size_t)64 * 128);
        amh_status st;
        if ((st = dalloc(c, (void **)&N->part, cap * 4)) != AMH_OK) return st;
        if ((st = dalloc(c, (void **)&N->bpart, capb * 4)) != AMH_OK) return st;
        N->part_cap = cap;
        N->bpart_cap = capb;
    }
    WgradArgs wa;
    wa.x = x;
    wa.g = g;
    wa.part = N->part;
    wa.bpart = N->bpart;
    wa.n = n;
    wa.h = h;
    wa.w = w;
    wa.cin = l.cin;
    wa.cout_pad = l.cout_pad;
    wa.kpad = l.kpad;
    wa.ks = l.ks;
    wa.chunk = chunk;
    HIPCHK(c, launch_wgrad(wa, N->g32 + l.w_off, N->g32 + l.b_off, splits, c->stream));
    if (dx) {
        // input gradient = convolution of g with the transposed, mirrored weights
        const int kpad_t = round_up(l.ks * l.ks * l.cout_pad, 32);
        HIPCHK(c, launch_transpose_w(N->pb + l.w_off, l.cin, l.cout_pad, l.kpad, l.ks, N->wt, kpad_t, c->stream));
        ConvArgs a;
        a.x = g;
        a.wgt = N->wt;
        a.bias = nullptr;
        a.mask = mask;
        a.y = dx;
        a.n = n;
        a.h = h;
        a.w = w;
        a.cin = l.cout_pad;
        a.cout_pad = l.cin;
        a.kpad = kpad_t;
        a.ks = l.ks;
        a.relu = 0;
        a.out_f32 = 0;
        HIPCHK(c, launch_conv(a, c->stream));
    }
    return AMH_OK;
}

DepthHead depth_head(const amh_params &p) {
    DepthHead dh;
    dh.d_min = p.depth_min;
    dh.d_max = p.depth_max;
    const double qf = 1.0 / (double)p.depth_max, qn = 1.0 / (double)p.depth_min;
    dh.q_far = (float)qf;
    dh.q_near = (float)qn;
    dh.R = (float)((qn - qf) / 12.0);
    return dh;
}

amh_status check_net(amh_ctx *c) {
    if (!c->net) return fail(c, AMH_E_STATE, "no proposal network (amh_nn_init or amh_nn_load)");
    return AMH_OK;
}

}  // namespace

namespace amh {

amh_status nn_reserve(amh_ctx *c, size_t cells) { return ensure_acts(c, cells); }

// forward pass on stream s; activations must be reserved (no allocation or synchronisation here,
// so that it can be captured into a graph)
amh_status nn_forward_stream(amh_ctx *c, const void *feats, const float *q_ref, int n, int h, int w, float *out,
                             hipStream_t s) {
    NetState *N = c->net;
    if (!N) return fail(c, AMH_E_STATE, "no proposal network (amh_nn_init or amh_nn_load)");
    const size_t P0 = (size_t)n * h * w;
    if (P0 > N->cap_px) return fail(c, AMH_E_STATE, "network activations not reserved for %zu cells", P0);
    amh_status st;
    HIPCHK(c, hipMemcpyAsync(N->x, feats, P0 * kIn * sizeof(bf16_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(N->qref, q_ref, P0 * sizeof(float), hipMemcpyDeviceToDevice, s));
    const int h1 = h / 2, w1 = w / 2, h2 = h / 4, w2 = w / 4, h3 = h / 8, w3 = w / 8;
#define FWD(li, in, outb, hh, ww)                                                \
    if ((st = conv_fwd(c, li, in, outb, n, hh, ww, false, s)) != AMH_OK) return st
    FWD(ENC0A, N->x, N->e0a, h, w);
    FWD(ENC0B, N->e0a, N->e0, h, w);
    HIPCHK(c, launch_pool(N->e0, n, h1, w1, 16, N->p0, s));
    FWD(ENC1A, N->p0, N->e1a, h1, w1);
    FWD(ENC1B, N->e1a, N->e1, h1, w1);
    HIPCHK(c, launch_pool(N->e1, n, h2, w2, 32, N->p1, s));
    FWD(ENC2A, N->p1, N->e2a, h2, w2);
    FWD(ENC2B, N->e2a, N->e2, h2, w2);
    HIPCHK(c, launch_pool(N->e2, n, h3, w3, 48, N->p2, s));
    FWD(ENC3A, N->p2, N->e3a, h3, w3);
    FWD(ENC3B, N->e3a, N->e3, h3, w3);
    HIPCHK(c, launch_upcat(N->e3, 64, N->e2, 48, n, h2, w2, N->c2, s));
    FWD(DEC2, N->c2, N->d2, h2, w2);
    HIPCHK(c, launch_upcat(N->d2, 48, N->e1, 32, n, h1, w1, N->c1, s));
    FWD(DEC1, N->c1, N->d1, h1, w1);
    HIPCHK(c, launch_upcat(N->d1, 32, N->e0, 16, n, h, w, N->c0, s));
    FWD(DEC0, N->c0, N->d0, h, w);
#undef FWD
    if ((st = conv_fwd(c, HEAD, N->d0, N->z, n, h, w, true, s)) != AMH_OK) return st;
    if (out) HIPCHK(c, launch_decode(N->z, N->qref, (int)P0, depth_head(c->p), out, s));
    N->n = n;
    N->h = h;
    N->w = w;
    N->have_fwd = true;
    return AMH_OK;
}

}  // namespace amh

extern "C" {

amh_status amh_nn_param_count(int64_t *n) {
    if (!n) return AMH_E_INVALID_ARG;
    *n = canonical_count();
    return AMH_OK;
}

amh_status amh_nn_init(amh_ctx *c, uint64_t seed) {
    if (!c) return AMH_E_INVALID_ARG;
    amh_status st = create_net(c);
    if (st != AMH_OK) return st;
    NetState *N = c->net;
    std::vector<float> canon((size_t)canonical_count());
    HostNormal rng{seed * 0x2545F4914F6CDD1Dull + 0x1234567ull};
    size_t o = 0;
    for (int i = 0; i < kLayers; ++i) {
        const LayerSpec &l = kSpec[i];
        const int fan_in = l.ks * l.ks * l.cin;
        const double sd = std::sqrt(2.0 / fan_in) * (i == HEAD ? 0.1 : 1.0);
        for (int e = 0; e < l.cout * fan_in; ++e) canon[o++] = (float)(sd * rng.normal());
        for (int co = 0; co < l.cout; ++co) canon[o++] = (i == HEAD && co == 3) ? -1.f : 0.f;
    }
    std::vector<float> pad;
    pack(N, canon.data(), pad);
    return upload_params(c, pad);
}

amh_status amh_nn_get_params(amh_ctx *c, float *out, int64_t n) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!out || n != canonical_count()) return fail(c, AMH_E_INVALID_ARG, "need out and n = %lld", (long long)canonical_count());
    amh_status st = check_net(c);
    if (st != AMH_OK) return st;
    std::vector<float> pad(c->net->n_pad);
    HIPCHK(c, hipMemcpyAsync(pad.data(), c->net->p32, pad.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unpack(c->net, pad, out);
    return AMH_OK;
}

amh_status amh_nn_set_params(amh_ctx *c, const float *in, int64_t n) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!in || n != canonical_count()) return fail(c, AMH_E_INVALID_ARG, "need in and n = %lld", (long long)canonical_count());
    amh_status st = create_net(c);
    if (st != AMH_OK) return st;
    std::vector<float> pad;
    pack(c->net, in, pad);
    return upload_params(c, pad);
}

amh_status amh_nn_get_grads(amh_ctx *c, float *out, int64_t n) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!out || n != canonical_count()) return fail(c, AMH_E_INVALID_ARG, "need out and n = %lld", (long long)canonical_count());
    amh_status st = check_net(c);
    if (st != AMH_OK) return st;
    if (!c->net->have_grad) return fail(c, AMH_E_STATE, "no gradient yet (amh_nn_backward)");
    std::vector<float> pad(c->net->n_pad);
    HIPCHK(c, hipMemcpyAsync(pad.data(), c->net->g32, pad.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    unpack(c->net, pad, out);
    return AMH_OK;
}

amh_status amh_nn_forward(amh_ctx *c, const void *feats, const float *q_ref, int n, int h, int w, float *out) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!q_ref) return fail(c, AMH_E_INVALID_ARG, "q_ref is NULL");
    if (!feats || n < 1 || h < 8 || w < 8 || h % 8 || w % 8 || (int64_t)n * h * w > (1ll << 28))
        return fail(c, AMH_E_INVALID_ARG, "need feats and n >= 1, h and w positive multiples of 8");
    amh_status st = check_net(c);
    if (st != AMH_OK) return st;
    if ((st = nn_reserve(c, (size_t)n * h * w)) != AMH_OK) return st;
    return nn_forward_stream(c, feats, q_ref, n, h, w, out, c->stream);
}

amh_status amh_nn_backward(amh_ctx *c, const float *target, float *loss) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!target) return fail(c, AMH_E_INVALID_ARG, "target is NULL");
    amh_status st = check_net(c);
    if (st != AMH_OK) return st;
    NetState *N = c->net;
    if (!N->have_fwd) return fail(c, AMH_E_STATE, "no forward pass to differentiate (amh_nn_forward)");
    const int n = N->n, h = N->h, w = N->w;
    const int P0 = n * h * w;
    const int h1 = h / 2, w1 = w / 2, h2 = h / 4, w2 = w / 4, h3 = h / 8, w3 = w / 8;
    hipStream_t s = c->stream;
    const int nb = loss_blocks(P0);
    if ((size_t)nb > N->loss_cap) {
        HIPCHK(c, hipStreamSynchronize(s));
        if (N->loss_part) (void)hipFree(N->loss_part);
        N->loss_part = nullptr;
        N->loss_cap = 0;
        if ((st = dalloc(c, (void **)&N->loss_part, (size_t)nb * 4)) != AMH_OK) return st;
        N->loss_cap = nb;
    }
    HIPCHK(c, launch_loss(N->z, N->qref, target, P0, depth_head(c->p), N->dz, N->loss_part, N->loss_dev, s));
#define BWD(li, x, g, dx, mask, hh, ww)                                          \
    if ((st = conv_bwd(c, li, x, g, dx, mask, n, hh, ww)) != AMH_OK) return st
    BWD(HEAD, N->d0, N->dz, N->g_d0, N->d0, h, w);          // dL/d(d0 pre-activation)
    BWD(DEC0, N->c0, N->g_d0, N->dc0, nullptr, h, w);        // dL/d(concat [up(d1), e0])
    HIPCHK(c, launch_up_grad(N->dc0, 48, N->d1, n, h1, w1, 32, N->g_d1, s));
    BWD(DEC1, N->c1, N->g_d1, N->dc1, nullptr, h1, w1);      // [up(d2), e1]
    HIPCHK(c, launch_up_grad(N->dc1, 80, N->d2, n, h2, w2, 48, N->g_d2, s));
    BWD(DEC2, N->c2, N->g_d2, N->dc2, nullptr, h2, w2);      // [up(e3), e2]
    HIPCHK(c, launch_up_grad(N->dc2, 112, N->e3, n, h3, w3, 64, N->g_e3, s));
    BWD(ENC3B, N->e3a, N->g_e3, N->g_e3a, N->e3a, h3, w3);
    BWD(ENC3A, N->p2, N->g_e3a, N->dp2, nullptr, h3, w3);
    HIPCHK(c, launch_enc_grad(N->dp2, N->dc2, 112, 64, N->e2, n, h2, w2, 48, N->g_e2, s));
    BWD(ENC2B, N->e2a, N->g_e2, N->g_e2a, N->e2a, h2, w2);
    BWD(ENC2A, N->p1, N->g_e2a, N->dp1, nullptr, h2, w2);
    HIPCHK(c, launch_enc_grad(N->dp1, N->dc1, 80, 48, N->e1, n, h1, w1, 32, N->g_e1, s));
    BWD(ENC1B, N->e1a, N->g_e1, N->g_e1a, N->e1a, h1, w1);
    BWD(ENC1A, N->p0, N->g_e1a, N->dp0, nullptr, h1, w1);
    HIPCHK(c, launch_enc_grad(N->dp0, N->dc0, 48, 32, N->e0, n, h, w, 16, N->g_e0, s));
    BWD(ENC0B, N->e0a, N->g_e0, N->g_e0a, N->e0a, h, w);
    BWD(ENC0A, N->x, N->g_e0a, nullptr, nullptr, h, w);
#undef BWD
    N->have_grad = true;
    if (loss) {
        HIPCHK(c, hipMemcpyAsync(loss, N->loss_dev, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return AMH_OK;
}

amh_status amh_nn_targets(amh_ctx *c, const float *depth, const float *normal, const float *cost, int width, int height,
                          float *target) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!depth || !normal || !cost || !target) return fail(c, AMH_E_INVALID_ARG, "depth, normal, cost and target are required");
    if (width < 1 || height < 1 || width > kMaxImageSide || height > kMaxImageSide)
        return fail(c, AMH_E_INVALID_ARG, "need 1 <= width, height <= %d", kMaxImageSide);
    const int h4 = 8 * ((height + 31) / 32), w4 = 8 * ((width + 31) / 32);
    HIPCHK(c, launch_targets(depth, normal, cost, width, height, kCell, h4, w4, c->p.beta, target, c->stream));
    return AMH_OK;
}

amh_status amh_nn_adam_step(amh_ctx *c, float lr, float beta1, float beta2, float eps) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
        !std::isfinite(lr))
        return fail(c, AMH_E_INVALID_ARG, "need lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
    amh_status st = check_net(c);
    if (st != AMH_OK) return st;
    NetState *N = c->net;
    if (!N->have_grad) return fail(c, AMH_E_STATE, "no gradient yet (amh_nn_backward)");
    ++N->step;
    HIPCHK(c, launch_adam(N->p32, N->g32, N->m, N->v, N->pb, (int)N->n_pad, lr, beta1, beta2, eps, N->step,
                          c->stream));
    N->have_fwd = false;  // the kept activations belong to the old parameters
    return AMH_OK;
}

amh_status amh_nn_save(amh_ctx *c, const char *path) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!path) return fail(c, AMH_E_INVALID_ARG, "path is NULL");
    const int64_t n = canonical_count();
    std::vector<float> canon((size_t)n);
    amh_status st = amh_nn_get_params(c, canon.data(), n);
    if (st != AMH_OK) return st;
    FILE *f = fopen(path, "wb");
    if (!f) return fail(c, AMH_E_INVALID_ARG, "cannot open %s for writing", path);
    const bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&n, 8, 1, f) == 1 &&
                    fwrite(canon.data(), 4, (size_t)n, f) == (size_t)n;
    if (fclose(f) != 0 || !ok) return fail(c, AMH_E_INVALID_ARG, "writing %s failed", path);
    return AMH_OK;
}

amh_status amh_nn_load(amh_ctx *c, const char *path) {
    if (!c) return AMH_E_INVALID_ARG;
    if (!path) return fail(c, AMH_E_INVALID_ARG, "path is NULL");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(c, AMH_E_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    int64_t n = 0;
    const int64_t want = canonical_count();
    std::vector<float> canon((size_t)want);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(&n, 8, 1, f) == 1 && n == want &&
              fread(canon.data(), 4, (size_t)n, f) == (size_t)n;
    fclose(f);
    if (!ok) return fail(c, AMH_E_INVALID_ARG, "%s is not a parameter file of this network (%lld floats)", path,
                         (long long)want);
    for (float v : canon)
        if (!std::isfinite(v)) return fail(c, AMH_E_INVALID_ARG, "%s holds non-finite parameters", path);
    return amh_nn_set_params(c, canon.data(), n);
}

}  // extern "C"
