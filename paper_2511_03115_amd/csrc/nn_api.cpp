// C ABI of the denoiser (declared in include/sde_nn.h): the network object
// (parameters, Adam state, activation and gradient buffers) and the
// sequence of kernel launches for inference, loss/gradient and update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "nn_internal.hpp"
#include "sde_nn.h"

using namespace sde;
using namespace sde::nn;

namespace {

#define NN_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return report_error(e_ == hipErrorOutOfMemory ? SDE_E_NOMEM : SDE_E_HIP,        \
                                (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

#define NN_CHECK(cond, msg)                                          \
    do {                                                             \
        if (!(cond)) return report_error(SDE_E_INVALID, (msg));      \
    } while (0)

// largest wgrad split-K partial buffer (floats)
constexpr long long kMaxPartFloats = 32LL << 20;

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

bool nt_ok(int co) {
    if (co % 16) return false;
    const int nt = co / 16;
    return nt == 1 || nt == 2 || nt == 3 || nt == 4 || nt == 6 || nt == 8 || nt == 12;
}

struct ConvP {
    long long w = 0, b = 0;   // offsets into the parameter vector
    int ci = 0, co = 0;
};

struct Level {
    uint16_t *ea = nullptr, *eb = nullptr, *pin = nullptr, *cat = nullptr, *da = nullptr,
             *db = nullptr;
    float *gE = nullptr, *gEa = nullptr, *gP = nullptr, *gCat = nullptr, *gDa = nullptr,
          *gDb = nullptr;
    // a split level's decoder conv input gradient (bf16), kept until the
    // encoder's pool_bwd into this level takes its skip half
    uint16_t* dzk = nullptr;
};

}  // namespace

struct sde_nn {
    sde_nn_config cfg{};
    int L = 0, c0 = 0, cin = 0;
    std::vector<int> c;
    std::vector<ConvP> enc_a, enc_b, dec_a, dec_b;   // dec_* indexed by level (L-1 entries)
    long long head_w = 0, head_b = 0, n_params = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    uint16_t* P16 = nullptr;
    long long step = 0;
    long long max_nv0 = 0;
    uint16_t* x16 = nullptr;    // input rows (training: the first weight gradient reads them)
    uint32_t* x2 = nullptr;     // the two used input channels as bf16 pairs
    float *resid = nullptr, *out = nullptr;
    std::vector<Level> lv;
    float *dout = nullptr, *loss_part = nullptr, *loss_dev = nullptr, *head_part = nullptr;
    uint16_t* dz = nullptr;
    uint16_t* dz2 = nullptr;      // the second bf16 output gradient of a 16 -> 16 chain
    uint16_t* wt_all = nullptr;   // every layer's flipped weights (offsets as in P16)
    float* wpart = nullptr;
    unsigned long long* maxbits = nullptr;
    std::vector<void*> allocs;
    bool have_grad = false;

    ~sde_nn() {
        for (void* p : allocs) (void)hipFree(p);
    }
};

namespace {

template <class T>
hipError_t dalloc(sde_nn* n, T** p, long long count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)std::max<long long>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    n->allocs.push_back(q);
    *p = (T*)q;
    return hipSuccess;
}

void dims_at(const int* d0, int l, int* d) {
    d[0] = d0[0];
    d[1] = d0[1] >> l;
    d[2] = d0[2] >> l;
    d[3] = d0[3] >> l;
}

long long nvox(const int* d) { return (long long)d[0] * d[1] * d[2] * d[3]; }

int check_dims(const sde_nn* n, int B, int D, int H, int W) {
    const int m = 1 << (n->L - 1);
    NN_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1, "volume sizes must be positive");
    NN_CHECK(D % m == 0 && H % m == 0 && W % m == 0,
             "D, H, W must be multiples of 2^(levels-1)");
    NN_CHECK((long long)B * D * H * W <= n->max_nv0, "volume exceeds the network's buffers");
    return SDE_OK;
}

// conv + LeakyReLU into bf16
int conv_act(sde_nn* n, const uint16_t* x, const ConvP& cp, const int* d, uint16_t* y) {
    NN_TRY(conv_fwd(x, n->P16 + cp.w, n->P + cp.b, d, cp.ci, cp.co, n->cfg.leaky_alpha, 1, y,
                    nullptr, 0, library_stream()));
    return SDE_OK;
}

// The first conv reads the input's two used channels as bf16 pairs (16
// outputs); the Cx-channel rows are then needed only by training's weight
// gradient.
bool first_from_pairs(const sde_nn* n) { return n->enc_a[0].co == 16; }

// The input rows x16 are written when a conv reads them.
uint16_t* input_rows(sde_nn* n) { return n->cfg.train || !first_from_pairs(n) ? n->x16 : nullptr; }

// The decoder conv of level l reads the concatenation [skip, up(low)] in
// place (inference always where the conv supports it; training also needs
// the weight gradient to read it so); otherwise it is stored in lv[l].cat.
bool cat_in_place(const sde_nn* n, int l, const int* d) {
    const ConvP& cp = n->dec_a[l];
    return !n->cfg.store_concat && conv_cat_fwd_supported(n->c[l], n->c[l + 1], cp.co, nvox(d)) &&
           (!n->cfg.train || wgrad_cat_supported(n->c[l], n->c[l + 1], cp.co, d));
}

int run_forward(sde_nn* n, const int* d0) {
    hipStream_t s = library_stream();
    int d[4], dc[4];
    // the pool after a 16 -> 16 second conv is fused into that conv
    auto pool_fused = [&](int l) {
        return l + 1 < n->L && n->enc_b[l].ci == 16 && n->enc_b[l].co == 16;
    };
    for (int l = 0; l < n->L; ++l) {
        dims_at(d0, l, d);
        Level& v = n->lv[l];
        const uint16_t* in = n->x16;
        if (l > 0) {
            if (!pool_fused(l - 1)) NN_TRY(pool_fwd(n->lv[l - 1].eb, d, n->c[l - 1], v.pin, s));
            in = v.pin;
        }
        if (l == 0 && first_from_pairs(n)) {
            const ConvP& cp = n->enc_a[0];
            NN_TRY(conv_in_fwd(n->x2, n->P16 + cp.w, n->cin, n->P + cp.b, d, n->cfg.leaky_alpha,
                               v.ea, s));
        } else if (int r = conv_act(n, in, n->enc_a[l], d, v.ea)) {
            return r;
        }
        if (pool_fused(l)) {
            const ConvP& cb = n->enc_b[l];
            NN_TRY(conv_pool_fwd(v.ea, n->P16 + cb.w, n->P + cb.b, d, n->cfg.leaky_alpha, v.eb,
                                 n->lv[l + 1].pin, s));
        } else if (int r = conv_act(n, v.ea, n->enc_b[l], d, v.eb)) {
            return r;
        }
    }
    const uint16_t* top = n->lv[n->L - 1].eb;
    for (int l = n->L - 2; l >= 0; --l) {
        dims_at(d0, l, d);
        dims_at(d0, l + 1, dc);
        (void)dc;
        Level& v = n->lv[l];
        const int Cf = n->c[l] + n->c[l + 1];
        const ConvP& cp = n->dec_a[l];
        if (cat_in_place(n, l, d)) {
            NN_TRY(conv_cat_fwd(v.eb, top, n->P16 + cp.w, n->P + cp.b, d, n->c[l], n->c[l + 1],
                                cp.co, n->cfg.leaky_alpha, 1, v.da, s));
        } else {
            NN_TRY(copy_channels(v.eb, d, n->c[l], Cf, 0, v.cat, s));
            NN_TRY(up_fwd(top, d, n->c[l + 1], Cf, n->c[l], v.cat, s));
            if (int r = conv_act(n, v.cat, cp, d, v.da)) return r;
        }
        const ConvP& cb = n->dec_b[l];
        if (l == 0 && cb.ci == 16 && cb.co == 16) {
            // the head fused into the last conv; inference does not keep its
            // activation
            NN_TRY(conv_head_fwd(v.da, n->P16 + cb.w, n->P + cb.b, d, n->cfg.leaky_alpha,
                                 n->cfg.train ? v.db : nullptr, n->P + n->head_w,
                                 n->P + n->head_b, n->resid, n->out, s));
            return SDE_OK;
        }
        if (int r = conv_act(n, v.da, cb, d, v.db)) return r;
        top = v.db;
    }
    NN_TRY(head_fwd(top, n->P + n->head_w, n->P + n->head_b, n->resid, nvox(d0), n->c0, n->out, s));
    return SDE_OK;
}

// backward through conv + LeakyReLU: weight/bias gradients into G; the
// gradient at the conv's output is dz_ready (bf16, already through the
// LeakyReLU derivative) when non-null, else lrelu_bwd(dy, y).  The input
// gradient goes (FP32) into dx when non-null, or, through the LeakyReLU
// derivative of the input activation y_in, (bf16) into dz_next when that is
// non-null (16 -> 16 convs).  The flipped weights are in n->wt_all (offset cp.w).
// With dz_up non-null the input gradient is split at channel cs: [0, cs)
// into dx, and [cs, ci), the upsampled half, through the upsampling backward
// and the LeakyReLU of the level below (activation y_up) into dz_up, bf16
// at half size (conv_fwd_split).  With x_low non-null the input is the
// concatenation [x (cs channels), up(x_low)] read in place.
int conv_bwd(sde_nn* n, const float* dy, const uint16_t* y, const uint16_t* x, const ConvP& cp,
             const int* d, float* dx, const uint16_t* dz_ready = nullptr,
             const uint16_t* y_in = nullptr, uint16_t* dz_next = nullptr, int cs = 0,
             const uint16_t* x_low = nullptr, const uint16_t* y_up = nullptr,
             uint16_t* dz_up = nullptr) {
    hipStream_t s = library_stream();
    const uint16_t* dz = dz_ready;
    if (!dz) {
        NN_TRY(lrelu_bwd(dy, y, n->cfg.leaky_alpha, nvox(d) * cp.co, n->dz, s));
        dz = n->dz;
    }
    const int chunk = wgrad_chunk_for(d, cp.ci, cp.co, kMaxPartFloats);
    if (x_low)
        NN_TRY(wgrad_cat(dz, x, x_low, d, cs, cp.ci - cs, cp.co, chunk, n->wpart, n->G + cp.w,
                         n->G + cp.b, s));
    else
        NN_TRY(wgrad(dz, x, d, cp.ci, cp.co, chunk, n->wpart, n->G + cp.w, n->G + cp.b, s));
    if (dz_next && cp.ci == 16 && cp.co == 16)
        NN_TRY(conv_dz_fwd(dz, n->wt_all + cp.w, d, y_in, n->cfg.leaky_alpha, dz_next, s));
    else if (dz_next)
        NN_TRY(conv_fwd(dz, n->wt_all + cp.w, nullptr, d, cp.co, cp.ci, n->cfg.leaky_alpha, 0,
                        dz_next, nullptr, 0, s, y_in));
    else if (dz_up)
        NN_TRY(conv_fwd_split(dz, n->wt_all + cp.w, d, cp.co, cp.ci, cs, dx, y_up,
                              n->cfg.leaky_alpha, dz_up, s));
    else if (dx)
        NN_TRY(conv_fwd(dz, n->wt_all + cp.w, nullptr, d, cp.co, cp.ci, 0.0f, 0, nullptr, dx, 0, s));
    return SDE_OK;
}

// A conv whose input gradient feeds only the LeakyReLU before it hands that
// layer its bf16 gradient directly: 16 -> 16 convs, and the wider ones whose
// input-gradient launch has the LeakyReLU-gradient epilogue at these dims.
bool dz_chain(const ConvP& cp, const int* d) {
    return (cp.ci == 16 && cp.co == 16) || conv_dz_wide_supported(cp.co, cp.ci, d);
}

// The decoder conv at level l whose input gradient conv_fwd_split takes:
// its skip half in FP32, its upsampled half straight to the level below as
// bf16 LeakyReLU gradient (no FP32 concatenation gradient at that level).
bool split_up(const sde_nn* n, int l) {
    return n->dec_b[l].ci == 16 && n->dec_b[l].co == 16 && n->dec_a[l].ci == 48 &&
           n->dec_a[l].co == 16 && n->c[l] == 16;
}

int run_backward(sde_nn* n, const int* d0) {
    hipStream_t s = library_stream();
    const int L = n->L;
    int d[4], dc[4];
    const long long nv0 = nvox(d0);
    const uint16_t* top0 = L > 1 ? n->lv[0].db : n->lv[0].eb;
    float* gtop0 = L > 1 ? n->lv[0].gDb : n->lv[0].gE;
    // every layer's flipped weights, in one launch
    FlipJobs fj;
    long long start = 0;
    for (auto* vec : {&n->enc_a, &n->enc_b, &n->dec_a, &n->dec_b})
        for (const ConvP& cp : *vec) {
            if (fj.n == kMaxFlipJobs) return SDE_E_INVALID;
            fj.w[fj.n] = n->P16 + cp.w;
            fj.wt[fj.n] = n->wt_all + cp.w;
            fj.ci[fj.n] = cp.ci;
            fj.co[fj.n] = cp.co;
            fj.start[fj.n] = start;
            start += 27LL * cp.ci * cp.co;
            ++fj.n;
        }
    fj.start[fj.n] = start;
    NN_TRY(flip_transpose_all(fj, s));
    // with a decoder, the head's input gradient feeds only the LeakyReLU of
    // the last conv: it is handed on as that conv's bf16 output gradient
    const bool head_dz = L > 1;
    NN_TRY(head_bwd(n->out /* holds dL/dout */, top0, n->P + n->head_w, nv0, n->c0, gtop0,
                    n->head_part, s, n->cfg.leaky_alpha, head_dz ? n->dz : nullptr));
    NN_TRY(sum_rows(n->head_part, head_bwd_blocks(nv0), n->c0 + 1, n->G + n->head_w, s));
    for (int l = 0; l <= L - 2; ++l) {
        dims_at(d0, l, d);
        dims_at(d0, l + 1, dc);
        Level& v = n->lv[l];
        const int Cf = n->c[l] + n->c[l + 1];
        // the output gradient of dec_b[l], through its LeakyReLU, already in
        // n->dz: from the head (level 0) or from the up_bwd of level l - 1
        const uint16_t* dzb = l == 0 ? (head_dz ? n->dz : nullptr) : n->dz;
        // the level below's output gradient: its only term, so it goes
        // through that layer's LeakyReLU, into n->dz for its conv_bwd
        float* tgt = (l + 1 <= L - 2) ? n->lv[l + 1].gDb : n->lv[L - 1].gE;
        const uint16_t* ytgt = (l + 1 <= L - 2) ? n->lv[l + 1].db : n->lv[L - 1].eb;
        const float al = n->cfg.leaky_alpha;
        // the level-0 decoder conv's input gradient: its upsampled half
        // goes through the upsampling backward and that LeakyReLU into n->dz;
        // its input, the conv's output gradient, is kept in v.dzk, and the
        // skip half is taken from it when the encoder reaches this level
        const bool split = split_up(n, l);
        uint16_t* dzd = split ? v.dzk : n->dz2;
        // the decoder conv's input: the stored concatenation, or the skip and
        // the level below read in place
        const bool inplace = cat_in_place(n, l, d);
        const uint16_t* low = l + 1 <= L - 2 ? n->lv[l + 1].db : n->lv[L - 1].eb;
        const uint16_t* xin = inplace ? v.eb : v.cat;
        const uint16_t* xlow = inplace ? low : nullptr;
        if (dz_chain(n->dec_b[l], d)) {
            if (int r = conv_bwd(n, v.gDb, v.db, v.da, n->dec_b[l], d, nullptr, dzb, v.da, dzd))
                return r;
            if (int r = conv_bwd(n, nullptr, nullptr, xin, n->dec_a[l], d, split ? nullptr : v.gCat,
                                 dzd, nullptr, nullptr, n->c[l], xlow, split ? ytgt : nullptr,
                                 split ? n->dz : nullptr))
                return r;
        } else {
            if (int r = conv_bwd(n, v.gDb, v.db, v.da, n->dec_b[l], d, v.gDa, dzb)) return r;
            if (int r = conv_bwd(n, v.gDa, v.da, xin, n->dec_a[l], d, v.gCat, nullptr, nullptr,
                                 nullptr, n->c[l], xlow))
                return r;
        }
        // the skip half stays in gCat, where the encoder's pool_bwd reads it
        if (!split) NN_TRY(up_bwd(v.gCat, dc, n->c[l + 1], Cf, n->c[l], tgt, s, ytgt, al, n->dz));
    }
    for (int l = L - 1; l >= 0; --l) {
        dims_at(d0, l, d);
        Level& v = n->lv[l];
        const uint16_t* in = l == 0 ? n->x16 : v.pin;
        // enc_b[l]'s output gradient, through its LeakyReLU, in n->dz: from
        // the decoder's last up_bwd (bottom level) or this level's pool_bwd
        // (which adds the pooled term to the skip term); a network of one
        // level has neither
        const uint16_t* dze = L > 1 ? n->dz : nullptr;
        if (dz_chain(n->enc_b[l], d)) {
            if (int r = conv_bwd(n, v.gE, v.eb, v.ea, n->enc_b[l], d, nullptr, dze, v.ea,
                                 n->dz2))
                return r;
            if (int r = conv_bwd(n, nullptr, nullptr, in, n->enc_a[l], d, l > 0 ? v.gP : nullptr,
                                 n->dz2))
                return r;
        } else {
            if (int r = conv_bwd(n, v.gE, v.eb, v.ea, n->enc_b[l], d, v.gEa, dze)) return r;
            if (int r = conv_bwd(n, v.gEa, v.ea, in, n->enc_a[l], d, l > 0 ? v.gP : nullptr))
                return r;
        }
        if (l > 0) {
            int df[4];
            dims_at(d0, l - 1, df);
            if (split_up(n, l - 1)) {
                // the skip half of the level's decoder conv input gradient
                // and the pooled term, through enc_b[l - 1]'s LeakyReLU
                NN_TRY(conv_dz_fwd(n->lv[l - 1].dzk, n->wt_all + n->dec_a[l - 1].w, df,
                                   n->lv[l - 1].eb, n->cfg.leaky_alpha, n->dz, s, v.gP));
            } else {
                // the skip term: the decoder's input gradient, channels
                // [0, c[l - 1]) of gCat
                NN_TRY(pool_bwd(v.gP, df, n->c[l - 1], n->lv[l - 1].gCat, s, n->lv[l - 1].eb,
                                n->cfg.leaky_alpha, n->dz, n->c[l - 1] + n->c[l]));
            }
        }
    }
    return SDE_OK;
}

int alloc_all(sde_nn* n) {
    const sde_nn_config& c = n->cfg;
    const int L = n->L;
    n->max_nv0 = (long long)c.max_batch * c.max_d * c.max_h * c.max_w;
    NN_TRY(dalloc(n, &n->P, n->n_params));
    NN_TRY(dalloc(n, &n->P16, n->n_params));
    NN_TRY(hipMemset(n->P, 0, sizeof(float) * n->n_params));
    NN_TRY(hipMemset(n->P16, 0, sizeof(uint16_t) * n->n_params));
    if (c.train || !first_from_pairs(n)) NN_TRY(dalloc(n, &n->x16, n->max_nv0 * n->cin));
    NN_TRY(dalloc(n, &n->x2, n->max_nv0));
    NN_TRY(dalloc(n, &n->resid, n->max_nv0));
    NN_TRY(dalloc(n, &n->out, n->max_nv0));
    NN_TRY(dalloc(n, &n->maxbits, 1));
    n->lv.assign(L, Level{});
    for (int l = 0; l < L; ++l) {
        const long long nv = n->max_nv0 >> (3 * l);
        Level& v = n->lv[l];
        NN_TRY(dalloc(n, &v.ea, nv * n->c[l]));
        NN_TRY(dalloc(n, &v.eb, nv * n->c[l]));
        if (l > 0) NN_TRY(dalloc(n, &v.pin, nv * n->c[l - 1]));
        if (l <= L - 2) {
            if (c.train || !conv_cat_fwd_supported(n->c[l], n->c[l + 1], n->c[l], nv))
                NN_TRY(dalloc(n, &v.cat, nv * (n->c[l] + n->c[l + 1])));
            NN_TRY(dalloc(n, &v.da, nv * n->c[l]));
            NN_TRY(dalloc(n, &v.db, nv * n->c[l]));
        }
        if (!c.train) continue;
        // above the bottom the skip gradient lives in gCat or is taken
        // from dzk: gE is the head's target (one level) or unused
        if (l <= L - 2 && split_up(n, l)) NN_TRY(dalloc(n, &v.dzk, nv * n->c[l]));
        else if (l == L - 1) NN_TRY(dalloc(n, &v.gE, nv * n->c[l]));
        NN_TRY(dalloc(n, &v.gEa, nv * n->c[l]));
        if (l > 0) NN_TRY(dalloc(n, &v.gP, nv * n->c[l - 1]));
        if (l <= L - 2) {
            if (!split_up(n, l)) NN_TRY(dalloc(n, &v.gCat, nv * (n->c[l] + n->c[l + 1])));
            NN_TRY(dalloc(n, &v.gDa, nv * n->c[l]));
            NN_TRY(dalloc(n, &v.gDb, nv * n->c[l]));
        }
    }
    if (!c.train) return SDE_OK;
    long long max_w = 0;
    for (auto* vec : {&n->enc_a, &n->enc_b, &n->dec_a, &n->dec_b})
        for (const ConvP& cp : *vec) max_w = std::max<long long>(max_w, 27LL * cp.ci * cp.co);
    NN_TRY(dalloc(n, &n->G, n->n_params));
    NN_TRY(dalloc(n, &n->M, n->n_params));
    NN_TRY(dalloc(n, &n->V, n->n_params));
    NN_TRY(hipMemset(n->G, 0, sizeof(float) * n->n_params));
    NN_TRY(hipMemset(n->M, 0, sizeof(float) * n->n_params));
    NN_TRY(hipMemset(n->V, 0, sizeof(float) * n->n_params));
    NN_TRY(dalloc(n, &n->dz, n->max_nv0 * n->c0));
    NN_TRY(dalloc(n, &n->dz2, n->max_nv0 * std::max(n->c0, 16)));
    NN_TRY(dalloc(n, &n->wt_all, n->n_params));
    NN_TRY(dalloc(n, &n->wpart, std::max(kMaxPartFloats, max_w)));
    NN_TRY(dalloc(n, &n->dout, n->max_nv0));
    NN_TRY(dalloc(n, &n->loss_part, mse_blocks(n->max_nv0)));
    NN_TRY(dalloc(n, &n->loss_dev, 1));
    NN_TRY(dalloc(n, &n->head_part, (long long)head_bwd_blocks(n->max_nv0) * (n->c0 + 1)));
    return SDE_OK;
}

}  // namespace

extern "C" {

int sde_nn_create(const sde_nn_config* cfg, sde_nn** out) {
    NN_CHECK(cfg && out, "null argument");
    *out = nullptr;
    const sde_nn_config& c = *cfg;
    NN_CHECK(c.levels >= 1 && c.levels <= 5, "levels must be 1..5");
    NN_CHECK(c.base_channels == 16 || c.base_channels == 32, "base_channels must be 16 or 32");
    NN_CHECK(c.in_channels >= 16 && c.in_channels % 16 == 0, "in_channels must be a multiple of 16");
    NN_CHECK(c.leaky_alpha > 0.0f, "leaky_alpha must be positive");
    NN_CHECK(c.max_batch >= 1 && c.max_d >= 1 && c.max_h >= 1 && c.max_w >= 1,
             "maximum sizes must be positive");
    const int m = 1 << (c.levels - 1);
    NN_CHECK(c.max_d % m == 0 && c.max_h % m == 0 && c.max_w % m == 0,
             "maximum D, H, W must be multiples of 2^(levels-1)");
    sde_nn* n = new sde_nn();
    n->cfg = c;
    n->L = c.levels;
    n->c0 = c.base_channels;
    n->cin = c.in_channels;
    for (int l = 0; l < n->L; ++l) n->c.push_back(n->c0 << l);
    long long off = 0;
    auto conv = [&](int ci, int co) {
        ConvP p;
        p.ci = ci;
        p.co = co;
        p.w = off;
        off += 27LL * ci * co;
        p.b = off;
        off += co;
        return p;
    };
    n->dec_a.resize(std::max(0, n->L - 1));
    n->dec_b.resize(std::max(0, n->L - 1));
    for (int l = 0; l < n->L; ++l) {
        n->enc_a.push_back(conv(l == 0 ? n->cin : n->c[l - 1], n->c[l]));
        n->enc_b.push_back(conv(n->c[l], n->c[l]));
    }
    for (int l = n->L - 2; l >= 0; --l) {
        n->dec_a[l] = conv(n->c[l] + n->c[l + 1], n->c[l]);
        n->dec_b[l] = conv(n->c[l], n->c[l]);
    }
    n->head_w = off;
    off += n->c0;
    n->head_b = off;
    off += 1;
    n->n_params = off;
    bool ok = true;
    for (auto* vec : {&n->enc_a, &n->enc_b, &n->dec_a, &n->dec_b})
        for (const ConvP& cp : *vec)
            ok = ok && nt_ok(cp.co) && nt_ok(cp.ci) && (cp.co / 16) * (cp.ci / 16) <= 64;
    if (!ok) {
        delete n;
        return report_error(SDE_E_INVALID, "channel counts outside the kernels' tile set");
    }
    n->cfg.adam_beta1 = c.adam_beta1 > 0 ? c.adam_beta1 : 0.9f;
    n->cfg.adam_beta2 = c.adam_beta2 > 0 ? c.adam_beta2 : 0.999f;
    n->cfg.adam_eps = c.adam_eps > 0 ? c.adam_eps : 1e-8f;
    if (int r = alloc_all(n)) {
        delete n;
        return r;
    }
    *out = n;
    return SDE_OK;
}

int sde_nn_destroy(sde_nn* net) {
    if (net) {
        (void)hipStreamSynchronize(library_stream());
        delete net;
    }
    return SDE_OK;
}

int sde_nn_param_count(const sde_nn* net, int64_t* n_out) {
    NN_CHECK(net && n_out, "null argument");
    *n_out = net->n_params;
    return SDE_OK;
}

int sde_nn_set_params(sde_nn* net, const float* params, int64_t n) {
    NN_CHECK(net && params, "null argument");
    NN_CHECK(n == net->n_params, "parameter count mismatch");
    hipStream_t s = library_stream();
    NN_TRY(hipMemcpyAsync(net->P, params, sizeof(float) * n, hipMemcpyHostToDevice, s));
    NN_TRY(f32_to_bf16(net->P, n, net->P16, s));
    NN_TRY(hipStreamSynchronize(s));
    return SDE_OK;
}

int sde_nn_get_params(sde_nn* net, float* params, int64_t n) {
    NN_CHECK(net && params, "null argument");
    NN_CHECK(n == net->n_params, "parameter count mismatch");
    hipStream_t s = library_stream();
    NN_TRY(hipMemcpyAsync(params, net->P, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    NN_TRY(hipStreamSynchronize(s));
    return SDE_OK;
}

int sde_nn_set_adam_state(sde_nn* net, const float* m, const float* v, int64_t n, int64_t step) {
    NN_CHECK(net && m && v, "null argument");
    NN_CHECK(net->cfg.train, "network was created without training buffers");
    NN_CHECK(n == net->n_params && step >= 0, "parameter count mismatch or negative step");
    hipStream_t s = library_stream();
    NN_TRY(hipMemcpyAsync(net->M, m, sizeof(float) * n, hipMemcpyHostToDevice, s));
    NN_TRY(hipMemcpyAsync(net->V, v, sizeof(float) * n, hipMemcpyHostToDevice, s));
    NN_TRY(hipStreamSynchronize(s));
    net->step = step;
    return SDE_OK;
}

int sde_nn_get_adam_state(sde_nn* net, float* m, float* v, int64_t n, int64_t* step) {
    NN_CHECK(net && m && v && step, "null argument");
    NN_CHECK(net->cfg.train, "network was created without training buffers");
    NN_CHECK(n == net->n_params, "parameter count mismatch");
    hipStream_t s = library_stream();
    NN_TRY(hipMemcpyAsync(m, net->M, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    NN_TRY(hipMemcpyAsync(v, net->V, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    NN_TRY(hipStreamSynchronize(s));
    *step = net->step;
    return SDE_OK;
}

int sde_nn_get_grads(sde_nn* net, float* grads, int64_t n) {
    NN_CHECK(net && grads, "null argument");
    NN_CHECK(net->cfg.train, "network was created without training buffers");
    NN_CHECK(n == net->n_params, "parameter count mismatch");
    hipStream_t s = library_stream();
    NN_TRY(hipMemcpyAsync(grads, net->G, sizeof(float) * n, hipMemcpyDeviceToHost, s));
    NN_TRY(hipStreamSynchronize(s));
    return SDE_OK;
}

int sde_nn_forward(sde_nn* net, const float* dose, const float* rho, int B, int D, int H, int W,
                   float* out) {
    NN_CHECK(net && dose && out, "null argument");
    if (int r = check_dims(net, B, D, H, W)) return r;
    const int d0[4] = {B, D, H, W};
    hipStream_t s = library_stream();
    NN_TRY(assemble_f32(dose, rho, nvox(d0), net->cin, input_rows(net), net->x2, net->resid, s));
    if (int r = run_forward(net, d0)) return r;
    NN_TRY(hipMemcpyAsync(out, net->out, sizeof(float) * nvox(d0), hipMemcpyDeviceToDevice, s));
    return SDE_OK;
}

int sde_nn_loss_grad(sde_nn* net, const float* dose, const float* rho, const float* target,
                     const float* weight, int B, int D, int H, int W, float* loss_out) {
    NN_CHECK(net && dose && target && loss_out, "null argument");
    NN_CHECK(net->cfg.train, "network was created without training buffers");
    if (int r = check_dims(net, B, D, H, W)) return r;
    const int d0[4] = {B, D, H, W};
    const long long nv0 = nvox(d0);
    hipStream_t s = library_stream();
    NN_TRY(assemble_f32(dose, rho, nv0, net->cin, input_rows(net), net->x2, net->resid, s));
    if (int r = run_forward(net, d0)) return r;
    // dL/dout overwrites the output buffer (the forward result is not kept)
    NN_TRY(mse(net->out, target, weight, nv0, net->out, net->loss_part, s));
    NN_TRY(sum_rows(net->loss_part, mse_blocks(nv0), 1, net->loss_dev, s));
    if (int r = run_backward(net, d0)) return r;
    NN_TRY(hipMemcpyAsync(loss_out, net->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s));
    NN_TRY(hipStreamSynchronize(s));
    net->have_grad = true;
    return SDE_OK;
}

int sde_nn_adam_step(sde_nn* net, float lr) {
    NN_CHECK(net, "null argument");
    NN_CHECK(net->cfg.train, "network was created without training buffers");
    NN_CHECK(net->have_grad, "no gradient: call sde_nn_loss_grad first");
    NN_CHECK(lr > 0.0f, "learning rate must be positive");
    net->step += 1;
    NN_TRY(adam(net->P, net->G, net->M, net->V, net->n_params, lr, net->cfg.adam_beta1,
                net->cfg.adam_beta2, net->cfg.adam_eps, (int)std::min<long long>(net->step, 1 << 30),
                net->P16, library_stream()));
    return SDE_OK;
}

int sde_nn_denoise(sde_nn* net, const double* dose, const float* rho, int nx, int ny, int nz,
                   double* out) {
    NN_CHECK(net && dose && out, "null argument");
    NN_CHECK(nx >= 1 && ny >= 1 && nz >= 1, "grid sizes must be positive");
    const int m = 1 << (net->L - 1);
    const int D = (nz + m - 1) / m * m, H = (ny + m - 1) / m * m, W = (nx + m - 1) / m * m;
    if (int r = check_dims(net, 1, D, H, W)) return r;
    const int d0[4] = {1, D, H, W};
    const int src[3] = {nz, ny, nx}, dst[3] = {D, H, W};
    hipStream_t s = library_stream();
    NN_TRY(fill_u32((uint32_t*)net->maxbits, 2, 0u, s));
    NN_TRY(max_abs(dose, (long long)nx * ny * nz, net->maxbits, s));
    const double* maxp = (const double*)net->maxbits;
    NN_TRY(assemble_grid(dose, rho, src, dst, maxp, net->cin, input_rows(net), net->x2, net->resid,
                         s));
    if (int r = run_forward(net, d0)) return r;
    NN_TRY(finish_grid(net->out, src, dst, maxp, out, s));
    return SDE_OK;
}

int sde_nn_prepare_pair(sde_nn* net, const double* low, const double* high, int64_t n, float eps,
                        float thr, float* low_out, float* high_out, float* weight_out) {
    NN_CHECK(net && low && low_out, "null argument");
    NN_CHECK(n >= 1, "size must be positive");
    NN_CHECK(!high || high_out, "high needs high_out");
    NN_CHECK(!weight_out || (high && eps > 0.0f && thr > 0.0f),
             "weight needs high, eps > 0 and thr > 0");
    hipStream_t s = library_stream();
    NN_TRY(fill_u32((uint32_t*)net->maxbits, 2, 0u, s));
    NN_TRY(max_abs(low, n, net->maxbits, s));
    NN_TRY(prepare_pair(low, high, n, (const double*)net->maxbits, eps, thr, low_out, high_out,
                        weight_out, s));
    return SDE_OK;
}

int sde_nn_conv3d_fwd(const uint16_t* x, const uint16_t* w, const float* bias, int B, int D,
                      int H, int W, int Ci, int Co, float alpha, int act, uint16_t* y16,
                      float* y32) {
    NN_CHECK(x && w && (y16 || y32), "null argument");
    NN_CHECK(aligned16(x) && aligned16(w) && aligned16(y16), "bf16 arrays must be 16-byte aligned");
    NN_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1, "volume sizes must be positive");
    NN_CHECK(Ci >= 16 && Ci % 16 == 0 && nt_ok(Co), "unsupported channel counts");
    const int d[4] = {B, D, H, W};
    NN_TRY(conv_fwd(x, w, bias, d, Ci, Co, alpha, act ? 1 : 0, y16, y32, 0, library_stream()));
    return SDE_OK;
}

int sde_nn_conv3d_workspace(int B, int D, int H, int W, int Ci, int Co, size_t* bytes) {
    NN_CHECK(bytes, "null argument");
    NN_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1, "volume sizes must be positive");
    NN_CHECK(Ci >= 16 && Ci % 16 == 0 && Co >= 16 && Co % 16 == 0, "unsupported channel counts");
    const int d[4] = {B, D, H, W};
    const long long wfl = 27LL * Ci * Co;
    const int chunk = wgrad_chunk_for(d, Ci, Co, kMaxPartFloats);
    const long long part = wgrad_part_floats(d, Ci, Co, chunk) * (long long)sizeof(float);
    *bytes = (size_t)std::max<long long>(part, wfl * (long long)sizeof(uint16_t));
    return SDE_OK;
}

int sde_nn_conv3d_dgrad(const uint16_t* dz, const uint16_t* w, int B, int D, int H, int W, int Ci,
                        int Co, float* dx, void* workspace, size_t workspace_bytes) {
    NN_CHECK(dz && w && dx && workspace, "null argument");
    NN_CHECK(aligned16(dz) && aligned16(w) && aligned16(workspace),
             "bf16 arrays and the workspace must be 16-byte aligned");
    NN_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1, "volume sizes must be positive");
    NN_CHECK(Co >= 16 && Co % 16 == 0 && nt_ok(Ci), "unsupported channel counts");
    NN_CHECK(workspace_bytes >= 27ULL * Ci * Co * sizeof(uint16_t), "workspace too small");
    const int d[4] = {B, D, H, W};
    hipStream_t s = library_stream();
    uint16_t* wt = (uint16_t*)workspace;
    NN_TRY(flip_transpose(w, wt, Ci, Co, s));
    NN_TRY(conv_fwd(dz, wt, nullptr, d, Co, Ci, 0.0f, 0, nullptr, dx, 0, s));
    return SDE_OK;
}

int sde_nn_conv3d_wgrad(const uint16_t* dz, const uint16_t* x, int B, int D, int H, int W, int Ci,
                        int Co, float* dw, float* db, void* workspace, size_t workspace_bytes) {
    NN_CHECK(dz && x && dw && workspace, "null argument");
    NN_CHECK(aligned16(dz) && aligned16(x) && aligned16(workspace),
             "bf16 arrays and the workspace must be 16-byte aligned");
    NN_CHECK(B >= 1 && D >= 1 && H >= 1 && W >= 1, "volume sizes must be positive");
    NN_CHECK(Ci >= 16 && Ci % 16 == 0 && Co >= 16 && Co % 16 == 0 &&
                 (Co / 16) * (Ci / 16) <= 64,
             "unsupported channel counts");
    size_t need = 0;
    if (int r = sde_nn_conv3d_workspace(B, D, H, W, Ci, Co, &need)) return r;
    NN_CHECK(workspace_bytes >= need, "workspace too small");
    const int d[4] = {B, D, H, W};
    const int chunk = wgrad_chunk_for(d, Ci, Co, kMaxPartFloats);
    NN_TRY(wgrad(dz, x, d, Ci, Co, chunk, (float*)workspace, dw, db, library_stream()));
    return SDE_OK;
}

}  // extern "C"
