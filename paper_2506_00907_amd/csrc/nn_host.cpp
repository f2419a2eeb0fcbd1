// Host side of the warm-start network (lbm_nn_* of lbm.h): the layer table of
// a three-level convolutional encoder-decoder, its device buffer layout, and
// the forward pass, backward pass and Adam update as sequences of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "nn_internal.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// activation tensors (index into the tensor table)
enum {
    T_IN, T_E1A, T_E1B, T_P1, T_E2A, T_E2B, T_P2, T_E3A, T_E3B, T_U2, T_D2A, T_D2B, T_U1, T_D1A, T_D1B, T_COUNT
};

struct Tensor {
    int level, ch;       // resolution level (size >> level) and channels
    size_t off = 0;      // element-type activations (buffer 2)
    size_t goff = 0;     // FP32 gradient (buffer 2), when it has one
    bool grad = true;
};

struct Layer {
    int in, out;                // tensors
    int cin, cout;              // real channels (master weights)
    int cinp, coutp;            // channels of the device tensors / padded output channels
    int taps, relu;
    size_t w_off, b_off;        // master parameters (FP32, buffer 0)
    size_t wf_off, wb_off;      // compute weights (buffer 1, element type)
};

struct Net {
    lbm_nn_desc d;
    std::vector<Tensor> t;
    std::vector<Layer> L;
    int64_t np = 0;             // parameters
    size_t wbytes = 0;          // compute weights
    size_t act_bytes = 0;       // buffer 2
    size_t out_off = 0, gout_off = 0, dz_off = 0, dwt_off = 0;
    size_t dwt_max = 0;
};

int64_t npix(const Net& n, int level, int N) {
    const int64_t s = n.d.size >> level;
    return (int64_t)N * s * s;
}

bool valid_desc(const lbm_nn_desc* d) {
    if (!d) return false;
    if (d->batch < 1 || d->size < 8 || d->size % 8) return false;
    if (d->in_ch < 1 || d->in_ch > 16 || d->out_ch < 1 || d->out_ch > 32) return false;
    if (d->width < 32 || d->width % 32) return false;
    if (d->precision != LBM_BF16 && d->precision != LBM_F32) return false;
    return true;
}

// layout of every buffer; returns false on an invalid description
bool build_net(const lbm_nn_desc* d, Net* n) {
    if (!valid_desc(d)) return false;
    n->d = *d;
    const int w = d->width;
    const size_t eb = d->precision == LBM_BF16 ? 2 : 4;
    n->t.assign(T_COUNT, Tensor{});
    auto T = [&](int id, int level, int ch, bool grad = true) {
        n->t[id].level = level;
        n->t[id].ch = ch;
        n->t[id].grad = grad;
    };
    T(T_IN, 0, 16, false);
    T(T_E1A, 0, w);
    T(T_E1B, 0, w);
    T(T_P1, 1, w);
    T(T_E2A, 1, 2 * w);
    T(T_E2B, 1, 2 * w);
    T(T_P2, 2, 2 * w);
    T(T_E3A, 2, 4 * w);
    T(T_E3B, 2, 4 * w);
    T(T_U2, 1, 6 * w);
    T(T_D2A, 1, 2 * w);
    T(T_D2B, 1, 2 * w);
    T(T_U1, 0, 3 * w);
    T(T_D1A, 0, w);
    T(T_D1B, 0, w);
    n->L.clear();
    auto C = [&](int in, int out, int cin, int cout, int taps, int relu) {
        Layer l;
        l.in = in;
        l.out = out;
        l.cin = cin;
        l.cout = cout;
        l.cinp = n->t[in].ch;
        l.coutp = out >= 0 ? n->t[out].ch : 32;
        l.taps = taps;
        l.relu = relu;
        n->L.push_back(l);
    };
    C(T_IN, T_E1A, d->in_ch, w, 9, 1);
    C(T_E1A, T_E1B, w, w, 9, 1);
    C(T_P1, T_E2A, w, 2 * w, 9, 1);
    C(T_E2A, T_E2B, 2 * w, 2 * w, 9, 1);
    C(T_P2, T_E3A, 2 * w, 4 * w, 9, 1);
    C(T_E3A, T_E3B, 4 * w, 4 * w, 9, 1);
    C(T_U2, T_D2A, 6 * w, 2 * w, 9, 1);
    C(T_D2A, T_D2B, 2 * w, 2 * w, 9, 1);
    C(T_U1, T_D1A, 3 * w, w, 9, 1);
    C(T_D1A, T_D1B, w, w, 9, 1);
    C(T_D1B, -1, w, d->out_ch, 1, 0);  // head: 1x1, linear, FP32 output
    // master parameters: per layer W[cout][cin][taps], then b[cout]
    int64_t np = 0;
    size_t wb = 0, dwt = 0;
    for (auto& l : n->L) {
        l.w_off = (size_t)np;
        np += (int64_t)l.cout * l.cin * l.taps;
        l.b_off = (size_t)np;
        np += l.cout;
        const size_t nw = (size_t)l.taps * l.coutp * l.cinp;
        l.wf_off = wb;
        wb += round_up(nw * eb, kAlign);
        l.wb_off = wb;
        wb += round_up(nw * eb, kAlign);
        dwt = std::max(dwt, nw);
    }
    n->np = np;
    n->wbytes = wb;
    n->dwt_max = dwt;
    // activations, gradients and scratch at the full batch
    const int N = d->batch;
    size_t o = 0;
    size_t dz = 0;
    for (auto& t : n->t) {
        const size_t cnt = (size_t)npix(*n, t.level, N) * t.ch;
        t.off = o;
        o += round_up(cnt * eb, kAlign);
        if (t.grad) {
            t.goff = o;
            o += round_up(cnt * 4, kAlign);
        }
    }
    for (auto& l : n->L) dz = std::max(dz, (size_t)npix(*n, l.out >= 0 ? n->t[l.out].level : 0, N) * l.coutp);
    n->out_off = o;
    o += round_up((size_t)npix(*n, 0, N) * d->out_ch * 4, kAlign);
    n->gout_off = o;
    o += round_up((size_t)npix(*n, 0, N) * 32 * 4, kAlign);
    n->dz_off = o;
    o += round_up(dz * eb, kAlign);
    n->dwt_off = o;
    o += round_up(dwt * 4, kAlign);
    n->act_bytes = o;
    return true;
}

void sizes_of(const Net& n, size_t s[4]) {
    s[0] = round_up((size_t)n.np * 4, kAlign) * 4;  // parameters, gradients, Adam m and v
    s[1] = n.wbytes;
    s[2] = n.act_bytes;
    s[3] = kAlign;  // loss accumulator
}

}  // namespace

struct lbm_nn {
    Net net;
    nnk::NnKernels k;
    void* buf[4];
    hipStream_t stream;
    int last_n = 0;        // batch of the last forward
    int64_t adam_t = 0;
    bool have_params = false;
    std::string err;
    float* P() const { return (float*)buf[0]; }
    float* G() const { return (float*)((char*)buf[0] + round_up((size_t)net.np * 4, kAlign)); }
    float* M() const { return (float*)((char*)buf[0] + 2 * round_up((size_t)net.np * 4, kAlign)); }
    float* V() const { return (float*)((char*)buf[0] + 3 * round_up((size_t)net.np * 4, kAlign)); }
    void* act(int id) const { return (char*)buf[2] + net.t[id].off; }
    float* grad(int id) const { return (float*)((char*)buf[2] + net.t[id].goff); }
};

namespace {

lbm_status nset(lbm_nn* n, lbm_status s, const std::string& m) {
    if (n) n->err = m;
    return s;
}

lbm_status nhip(lbm_nn* n, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    return nset(n, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NN_CHECK(expr, what)                               \
    do {                                                   \
        lbm_status _s = nhip(n, (expr), what);             \
        if (_s != LBM_OK) return _s;                       \
    } while (0)

lbm_status prep_weights(lbm_nn* n) {
    for (const auto& l : n->net.L)
        NN_CHECK(n->k.prep(n->P() + l.w_off, l.cout, l.cin, l.coutp, l.cinp, l.taps, (char*)n->buf[1] + l.wf_off,
                           (char*)n->buf[1] + l.wb_off, n->stream),
                 "weight preparation");
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_nn_required_bytes(const lbm_nn_desc* d, size_t sizes_out[4]) {
    Net n;
    if (!build_net(d, &n)) return 0;
    size_t s[4];
    sizes_of(n, s);
    size_t tot = 0;
    for (int i = 0; i < 4; ++i) {
        if (sizes_out) sizes_out[i] = s[i];
        tot += s[i];
    }
    return tot;
}

lbm_status lbm_nn_create(const lbm_nn_desc* d, void* const dev_bufs[4], void* hip_stream, lbm_nn** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    Net net;
    if (!build_net(d, &net) || !dev_bufs) return LBM_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!dev_bufs[i] || ((uintptr_t)dev_bufs[i] % kAlign) != 0) return LBM_EINVAL;
    lbm_nn* n = new lbm_nn();
    n->net = net;
    n->k = d->precision == LBM_BF16 ? nnk::nn_kernels_bf16() : nnk::nn_kernels_f32();
    for (int i = 0; i < 4; ++i) n->buf[i] = dev_bufs[i];
    n->stream = (hipStream_t)hip_stream;
    *out = n;
    return LBM_OK;
}

int64_t lbm_nn_num_params(const lbm_nn* n) { return n ? n->net.np : -1; }

lbm_status lbm_nn_set_params(lbm_nn* n, const float* dev_params) {
    if (!n) return LBM_EINVAL;
    if (!dev_params) return nset(n, LBM_EINVAL, "params is NULL");
    const int64_t np = n->net.np;
    NN_CHECK(hipMemcpyAsync(n->P(), dev_params, (size_t)np * 4, hipMemcpyDeviceToDevice, n->stream), "param copy");
    NN_CHECK(nnk::nn_fill(n->M(), np, 0.f, n->stream), "moment clear");
    NN_CHECK(nnk::nn_fill(n->V(), np, 0.f, n->stream), "moment clear");
    NN_CHECK(nnk::nn_fill(n->G(), np, 0.f, n->stream), "gradient clear");
    n->adam_t = 0;
    lbm_status st = prep_weights(n);
    if (st) return st;
    n->have_params = true;
    return LBM_OK;
}

lbm_status lbm_nn_get_params(lbm_nn* n, float* dev_out) {
    if (!n || !dev_out) return LBM_EINVAL;
    NN_CHECK(hipMemcpyAsync(dev_out, n->P(), (size_t)n->net.np * 4, hipMemcpyDeviceToDevice, n->stream), "param copy");
    return LBM_OK;
}

lbm_status lbm_nn_get_grads(lbm_nn* n, float* dev_out) {
    if (!n || !dev_out) return LBM_EINVAL;
    NN_CHECK(hipMemcpyAsync(dev_out, n->G(), (size_t)n->net.np * 4, hipMemcpyDeviceToDevice, n->stream), "grad copy");
    return LBM_OK;
}

lbm_status lbm_nn_forward(lbm_nn* n, int32_t N, const float* dev_x, float* dev_y) {
    if (!n) return LBM_EINVAL;
    if (N < 1 || N > n->net.d.batch) return nset(n, LBM_EINVAL, "batch out of range");
    if (!dev_x) return nset(n, LBM_EINVAL, "input is NULL");
    if (!n->have_params) return nset(n, LBM_ESTATE, "lbm_nn_set_params must come first");
    const Net& net = n->net;
    const int S = net.d.size;
    hipStream_t s = n->stream;
    NN_CHECK(n->k.pack(dev_x, npix(net, 0, N), net.d.in_ch, 16, n->act(T_IN), s), "input pack");
    auto conv = [&](int li) -> lbm_status {
        const Layer& l = net.L[li];
        const int lv = net.t[l.in].level, sz = S >> lv;
        const void* Wf = (char*)n->buf[1] + l.wf_off;
        const float* b = n->P() + l.b_off;
        if (l.out >= 0)
            NN_CHECK(n->k.conv(n->act(l.in), Wf, b, N, sz, sz, l.cinp, l.coutp, l.coutp, l.taps, l.relu, n->act(l.out),
                               nullptr, 0, s),
                     "conv");
        else
            NN_CHECK(n->k.conv(n->act(l.in), Wf, b, N, sz, sz, l.cinp, l.coutp, net.d.out_ch, l.taps, 0, nullptr,
                               (float*)((char*)n->buf[2] + net.out_off), 0, s),
                     "head conv");
        return LBM_OK;
    };
    lbm_status st;
    const int w = net.d.width;
    if ((st = conv(0)) || (st = conv(1))) return st;
    NN_CHECK(n->k.pool(n->act(T_E1B), N, S, S, w, n->act(T_P1), s), "pool");
    if ((st = conv(2)) || (st = conv(3))) return st;
    NN_CHECK(n->k.pool(n->act(T_E2B), N, S / 2, S / 2, 2 * w, n->act(T_P2), s), "pool");
    if ((st = conv(4)) || (st = conv(5))) return st;
    NN_CHECK(n->k.upcat(n->act(T_E3B), n->act(T_E2B), N, S / 2, S / 2, 4 * w, 2 * w, n->act(T_U2), s), "upcat");
    if ((st = conv(6)) || (st = conv(7))) return st;
    NN_CHECK(n->k.upcat(n->act(T_D2B), n->act(T_E1B), N, S, S, 2 * w, w, n->act(T_U1), s), "upcat");
    if ((st = conv(8)) || (st = conv(9)) || (st = conv(10))) return st;
    n->last_n = N;
    if (dev_y)
        NN_CHECK(hipMemcpyAsync(dev_y, (char*)n->buf[2] + net.out_off, (size_t)npix(net, 0, N) * net.d.out_ch * 4,
                                hipMemcpyDeviceToDevice, s),
                 "output copy");
    return LBM_OK;
}

lbm_status lbm_nn_backward(lbm_nn* n, const float* dev_target, const float* dev_weight, double* host_loss) {
    if (!n) return LBM_EINVAL;
    if (!dev_target || !dev_weight) return nset(n, LBM_EINVAL, "target or weight is NULL");
    if (n->last_n < 1) return nset(n, LBM_ESTATE, "lbm_nn_forward must come first");
    const Net& net = n->net;
    const int N = n->last_n, S = net.d.size, w = net.d.width;
    hipStream_t s = n->stream;
    double* lossp = (double*)n->buf[3];
    float* gout = (float*)((char*)n->buf[2] + net.gout_off);
    void* dz = (char*)n->buf[2] + net.dz_off;
    float* dwt = (float*)((char*)n->buf[2] + net.dwt_off);
    NN_CHECK(nnk::nn_fill_f64(lossp, 1, s), "loss clear");
    NN_CHECK(nnk::nn_fill(n->G(), net.np, 0.f, s), "gradient clear");
    NN_CHECK(n->k.loss((const float*)((char*)n->buf[2] + net.out_off), dev_target, dev_weight, npix(net, 0, N),
                       net.d.out_ch, 32, gout, lossp, s),
             "loss");
    // one layer: dZ from the output gradient, weight and bias gradients, and
    // the input gradient (except for the first layer)
    auto back = [&](int li, const float* gy) -> lbm_status {
        const Layer& l = net.L[li];
        const int lv = net.t[l.in].level, sz = S >> lv;
        const int64_t np_ = npix(net, lv, N);
        const void* yact = l.out >= 0 ? n->act(l.out) : nullptr;
        NN_CHECK(n->k.act_grad(gy, yact, np_ * l.coutp, l.relu, dz, s), "activation gradient");
        NN_CHECK(nnk::nn_fill(dwt, (int64_t)l.taps * l.coutp * l.cinp, 0.f, s), "weight-gradient clear");
        NN_CHECK(n->k.wgrad(n->act(l.in), dz, N, sz, sz, l.cinp, l.coutp, l.taps, dwt, s), "weight gradient");
        NN_CHECK(n->k.gather(dwt, l.cout, l.cin, l.coutp, l.cinp, l.taps, n->G() + l.w_off, s), "gradient gather");
        NN_CHECK(n->k.bgrad(dz, np_, l.coutp, l.cout, n->G() + l.b_off, s), "bias gradient");
        if (li > 0)
            NN_CHECK(n->k.conv(dz, (char*)n->buf[1] + l.wb_off, nullptr, N, sz, sz, l.coutp, l.cinp, l.cinp, l.taps, 0,
                               nullptr, n->grad(l.in), 0, s),
                     "input gradient");
        return LBM_OK;
    };
    lbm_status st;
    if ((st = back(10, gout)) || (st = back(9, n->grad(T_D1B))) || (st = back(8, n->grad(T_D1A)))) return st;
    NN_CHECK(n->k.upcat_grad(n->grad(T_U1), N, S, S, 2 * w, w, n->grad(T_D2B), n->grad(T_E1B), s), "upcat gradient");
    if ((st = back(7, n->grad(T_D2B))) || (st = back(6, n->grad(T_D2A)))) return st;
    NN_CHECK(n->k.upcat_grad(n->grad(T_U2), N, S / 2, S / 2, 4 * w, 2 * w, n->grad(T_E3B), n->grad(T_E2B), s),
             "upcat gradient");
    if ((st = back(5, n->grad(T_E3B))) || (st = back(4, n->grad(T_E3A)))) return st;
    NN_CHECK(n->k.pool_grad(n->grad(T_P2), N, S / 2, S / 2, 2 * w, n->grad(T_E2B), s), "pool gradient");
    if ((st = back(3, n->grad(T_E2B))) || (st = back(2, n->grad(T_E2A)))) return st;
    NN_CHECK(n->k.pool_grad(n->grad(T_P1), N, S, S, w, n->grad(T_E1B), s), "pool gradient");
    if ((st = back(1, n->grad(T_E1B))) || (st = back(0, n->grad(T_E1A)))) return st;
    if (host_loss) {
        NN_CHECK(hipMemcpyAsync(host_loss, lossp, sizeof(double), hipMemcpyDeviceToHost, s), "loss copy");
        NN_CHECK(hipStreamSynchronize(s), "loss sync");
    }
    return LBM_OK;
}

lbm_status lbm_nn_adam_step(lbm_nn* n, float lr, float beta1, float beta2, float eps) {
    if (!n) return LBM_EINVAL;
    if (!n->have_params) return nset(n, LBM_ESTATE, "lbm_nn_set_params must come first");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return nset(n, LBM_EINVAL, "bad Adam hyper-parameters");
    n->adam_t++;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)n->adam_t));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)n->adam_t));
    NN_CHECK(nnk::nn_adam(n->P(), n->G(), n->M(), n->V(), n->net.np, lr, beta1, beta2, eps, bc1, bc2, n->stream),
             "adam");
    return prep_weights(n);
}

const char* lbm_nn_last_error(const lbm_nn* n) { return n ? n->err.c_str() : "null network"; }

void lbm_nn_destroy(lbm_nn* n) { delete n; }

}  // extern "C"
