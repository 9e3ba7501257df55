// C-ABI of the warm-start proxy kernels (declared in include/opf.h).
#include <cstdint>
#include <vector>

#include "internal.h"
#include "proxy_kernels.h"

using namespace opf_internal;

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool mult4(int v) { return v >= 0 && v % 4 == 0; }

int launched(hipError_t e, const char* what) { return e == hipSuccess ? OPF_OK : hip_err(e, what); }

int static_model(opf_model m) {
    if (!valid_model(m)) return set_err(OPF_E_STATE, "invalid or destroyed model handle");
    if (m->hm.ly.nrep != 1) return set_err(OPF_E_ARG, "the proxy kernels take a static model");
    if (m->hm.ly.rect) return set_err(OPF_E_ARG, "the proxy kernels take a polar model");
    return OPF_OK;
}

opf::ProxBox box_of(opf_model m, double va_span) {
    const opf::Layout& ly = m->hm.ly;
    opf::ProxBox b{};
    b.N = ly.N;
    b.G = ly.G;
    b.vmin = m->lvar + ly.x_vm;
    b.vmax = m->uvar + ly.x_vm;
    b.pmin = m->lvar + ly.x_pg;
    b.pmax = m->uvar + ly.x_pg;
    b.qmin = m->lvar + ly.x_qg;
    b.qmax = m->uvar + ly.x_qg;
    b.is_ref = m->is_ref;
    b.va_span = va_span;
    return b;
}

opf::ProxRows rows_of(opf_model m) {
    const opf::Layout& ly = m->hm.ly;
    opf::ProxRows r{};
    r.m = (int32_t)ly.m();
    r.n = (int32_t)ly.n;
    r.L = ly.L;
    r.flow0 = (int32_t)ly.c_blk[opf::B_PFR];
    r.flow1 = (int32_t)ly.c_blk[opf::B_ANG];
    r.pq0 = (int32_t)ly.x_p;
    r.npq = 4 * ly.L;
    r.thf = (int32_t)ly.c_blk[opf::B_THF];
    r.tht = (int32_t)ly.c_blk[opf::B_THT];
    r.balp = (int32_t)ly.c_blk[opf::B_BALP];
    r.balq = (int32_t)ly.c_blk[opf::B_BALQ];
    r.f_bus = m->dm.f_bus;
    r.t_bus = m->dm.t_bus;
    r.lcon = m->lcon;
    r.ucon = m->ucon;
    r.lvar = m->lvar;
    r.uvar = m->uvar;
    return r;
}

// The fused loss kernel's conditions beyond a static polar model: no storage
// units or devices, x in the order (va, vm, pg, qg, p, q), and one sample's
// working set within 64 KiB of LDS.
constexpr size_t kFusedLdsMax = 65536;
bool fused_fits(opf_model m) {
    const opf::Layout& ly = m->hm.ly;
    const int64_t N = ly.N, G = ly.G, L = ly.L;
    return ly.nrep == 1 && !ly.rect && ly.S == 0 && ly.D == 0 && ly.x_va == 0 && ly.x_vm == N &&
           ly.x_pg == 2 * N && ly.x_qg == 2 * N + G && ly.x_p == 2 * N + 2 * G && ly.x_q == ly.x_p + 2 * L &&
           opf::prox_loss_fused_lds(ly.N, ly.L, ly.G) <= kFusedLdsMax;
}


// The training step's workspace: every buffer of one step carved from the
// caller's block (256-byte aligned), and the per-layer operand choices of
// the autograd path (BF16 weights where a BF16 copy is kept and the input
// width is a multiple of 8; BF16 hidden activations where the width is).
struct TrainPlan {
    int nl = 0, B = 0, D = 0, chunks = 0, maxd = 0;
    std::vector<int64_t> wo, bo;                  // weight and bias offsets (floats)
    std::vector<int> fo, fi, splits;
    std::vector<bool> w_bf16, act_bf16;
    std::vector<size_t> pre, act;                 // byte offsets of each layer's pre-activation and activation
    size_t dz = 0, gflat = 0, cwork = 0, skw = 0, d0 = 0, d1 = 0, dt0 = 0, dt1 = 0, dh = 0, total = 0;
    int64_t n_params = 0;
};

int make_plan(const prox_mlp_desc* mlp, int B, TrainPlan& P) {
    if (!mlp || mlp->n_layers < 1 || !mlp->dims) return set_err(OPF_E_ARG, "bad MLP descriptor");
    if (B < 4 || B % 4) return set_err(OPF_E_ARG, "the batch must be a positive multiple of 4");
    P.nl = mlp->n_layers;
    P.B = B;
    P.chunks = (B + 127) / 128;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    int64_t par = 0;
    for (int k = 0; k <= P.nl; k++) {
        const int d = mlp->dims[k];
        if (d < 4 || d % 4) return set_err(OPF_E_ARG, "layer widths must be positive multiples of 4");
        P.maxd = std::max(P.maxd, d);
    }
    size_t sk = 4;
    for (int k = 0; k < P.nl; k++) {
        const int fi = mlp->dims[k], fo = mlp->dims[k + 1];
        P.fi.push_back(fi);
        P.fo.push_back(fo);
        P.wo.push_back(par);
        P.bo.push_back(par + (int64_t)fo * fi);
        par += (int64_t)fo * fi + fo;
        P.w_bf16.push_back(mlp->flat_bf16 != nullptr && fi % 8 == 0);
        if (P.w_bf16.back() && (P.wo.back() % 8 || !aligned16(mlp->flat_bf16)))  // the products' 16-byte loads
            return set_err(OPF_E_ARG, "layer %d's BF16 weights are not 16-byte aligned", k);
        P.act_bf16.push_back(k < P.nl - 1 && mlp->flat_bf16 != nullptr && fo % 8 == 0);
        const int sp = opf::prox_gemm_splits(fo, fi, B);
        P.splits.push_back(sp);
        if (sp > 1) sk = std::max(sk, (size_t)sp * fo * fi);
        P.pre.push_back(take(sizeof(float) * (size_t)B * fo));
        P.act.push_back(k < P.nl - 1 ? take((P.act_bf16.back() ? 2 : 4) * (size_t)B * fo) : 0);
    }
    P.n_params = par;
    P.D = mlp->dims[P.nl];
    P.dz = take(sizeof(float) * (size_t)B * P.D);
    P.gflat = take(sizeof(float) * (size_t)par);
    P.cwork = take(sizeof(float) * (size_t)P.chunks * P.maxd);
    P.skw = take(sizeof(float) * sk);
    P.d0 = take(sizeof(float) * (size_t)B * P.maxd);
    P.d1 = take(sizeof(float) * (size_t)B * P.maxd);
    P.dt0 = take(2 * (size_t)B * P.maxd);  // BF16, dpre transposed
    P.dt1 = take(2 * (size_t)B * P.maxd);
    P.dh = take(sizeof(float) * (size_t)B * P.maxd);
    P.total = off;
    return OPF_OK;
}

}  // namespace

extern "C" {

int prox_train_step_bytes(const prox_mlp_desc* mlp, int B, int64_t* bytes) {
    TrainPlan P;
    if (int rc = make_plan(mlp, B, P)) return rc;
    if (!bytes) return set_err(OPF_E_ARG, "bytes must be non-NULL");
    *bytes = (int64_t)P.total;
    return OPF_OK;
}

namespace {
// GPU-side phase marks of one training step (phase_ms != NULL only)
struct PhaseEvents {
    hipEvent_t ev[5] = {};
    int n = 0;
    bool on = false;
    hipError_t err = hipSuccess;  // the first failed record, reported when the times are read
    explicit PhaseEvents(bool want) : on(want) {
        if (!on) return;
        for (; n < 5; n++)
            if (hipEventCreate(&ev[n]) != hipSuccess) break;
        on = n == 5;
    }
    void mark(int i, hipStream_t s) {
        if (on && err == hipSuccess) err = hipEventRecord(ev[i], s);
    }
    ~PhaseEvents() {
        for (int i = 0; i < n; i++) (void)hipEventDestroy(ev[i]);  // nothing to report from a destructor
    }
};
}  // namespace

int prox_train_step(opf_model model, const prox_mlp_desc* mlp, const float* feats, const double* loads, int B,
                    double va_span, double rho, double obj_scale, float lr, float beta1, float beta2, float eps,
                    void* work, int64_t work_bytes, double* loss, double* cvio, float* phase_ms, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (!fused_fits(model)) return set_err(OPF_E_ARG, "the training step takes a model that prox_loss_fused takes");
    TrainPlan P;
    if (int rc = make_plan(mlp, B, P)) return rc;
    const opf::Layout& ly = model->hm.ly;
    if (P.D != 2 * ly.N + 2 * ly.G) return set_err(OPF_E_ARG, "the MLP's output width must be 2N + 2G");
    if (!feats || !loads || !loss || !cvio || !work || !mlp->flat || !mlp->m1 || !mlp->m2 || !mlp->step)
        return set_err(OPF_E_ARG, "bad arguments");
    if (!aligned16(feats) || !aligned16(work) || !aligned16(mlp->flat) || (mlp->flat_bf16 && !aligned16(mlp->flat_bf16)))
        return set_err(OPF_E_ARG, "feats, work and the parameters must be 16-byte aligned");
    if (work_bytes < (int64_t)P.total) return set_err(OPF_E_ARG, "work holds %lld bytes, the step needs %zu",
                                                      (long long)work_bytes, P.total);
    DeviceGuard dg(model->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    PhaseEvents pe(phase_ms != nullptr);
    if (phase_ms && !pe.on) return set_err(OPF_E_STATE, "could not create the phase events");
    pe.mark(0, s);
    char* W = static_cast<char*>(work);
    const float* flat = mlp->flat;
    const __bf16* fb = static_cast<const __bf16*>(mlp->flat_bf16);
    auto weight = [&](int k) -> const void* { return P.w_bf16[k] ? (const void*)(fb + P.wo[k]) : (const void*)(flat + P.wo[k]); };
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; return r == hipSuccess; };
    // forward: x W^T + b with GELU on the hidden layers (the activations BF16 where chosen)
    const void* h = feats;
    bool h_bf16 = false;
    for (int k = 0; k < P.nl; k++) {
        const bool hidden = k < P.nl - 1;
        if (!ok(opf::prox_gemm_mixed(0, h, h_bf16, P.fi[k], weight(k), P.w_bf16[k], P.fi[k],
                                     reinterpret_cast<float*>(W + P.pre[k]), P.fo[k], B, P.fo[k], P.fi[k],
                                     flat + P.bo[k], hidden ? W + P.act[k] : nullptr, hidden && P.act_bf16[k], 0, 1,
                                     nullptr, s)))
            return hip_err(e, "prox_train_step forward");
        if (hidden) {
            h = W + P.act[k];
            h_bf16 = P.act_bf16[k];
        }
    }
    pe.mark(1, s);
    // the loss with d loss / d z, then the mean's weight 1/B
    const float* z = reinterpret_cast<const float*>(W + P.pre[P.nl - 1]);
    float* dz = reinterpret_cast<float*>(W + P.dz);
    const opf::ProxPerm pm{model->he_pos, model->gen_pos};
    // d loss / d z scaled by the mean's 1/B and rounded to FP32 by the loss kernel itself, then the top
    // layer's bias sums' first pass over it
    if (!ok(opf::prox_loss_fused(model->dm, box_of(model, va_span), rows_of(model), pm, z, loads, B, rho, obj_scale,
                                 loss, cvio, nullptr, nullptr, nullptr, s, dz, 1.0 / B)) ||
        !ok(opf::prox_colsum_first(dz, B, P.D, reinterpret_cast<float*>(W + P.cwork), s)))
        return hip_err(e, "prox_train_step loss");
    pe.mark(2, s);
    // backward: weight gradients (split over the batch), bias column sums and
    // the GELU backward of the layer below in the dh product
    float* gflat = reinterpret_cast<float*>(W + P.gflat);
    float* cwork = reinterpret_cast<float*>(W + P.cwork);
    float* skw = reinterpret_cast<float*>(W + P.skw);
    const void* dpre = dz;
    const void* dpreT = nullptr;  // dpre transposed (BF16, [fo, B]) when the dh product wrote it
    bool d_bf16 = false, parts = true;  // the top layer's column sums' first pass came with dz
    char* dbuf[2] = {W + P.d0, W + P.d1};
    char* dtbuf[2] = {W + P.dt0, W + P.dt1};
    for (int k = P.nl - 1; k >= 0; k--) {
        const int fo = P.fo[k], fi = P.fi[k];
        const void* h_in = k == 0 ? (const void*)feats : (const void*)(W + P.act[k - 1]);
        const bool h_in_bf16 = k > 0 && P.act_bf16[k - 1];
        // dW = dpre^T h_in reads dpre k-contiguous from its transposed copy where there is one (the same
        // products in the same order, a faster operand load)
        const bool tr = dpreT != nullptr;
        const int wv = tr ? 1 : 2, wlda = tr ? B : fo;
        const void* wa = tr ? dpreT : dpre;
        const bool wa_bf16 = tr || d_bf16;
        if (P.splits[k] > 1 && parts) {
            // the split-K parts, then their sum and the bias sums' second pass in one launch
            if (!ok(opf::prox_gemm_split_parts(wv, wa, wa_bf16, wlda, h_in, h_in_bf16, fi, fo, fi, B, P.splits[k], skw,
                                               s)) ||
                !ok(opf::prox_wgrad_finish(skw, P.splits[k], fo, fi, gflat + P.wo[k], fi, cwork, P.chunks, fo,
                                           gflat + P.bo[k], s)))
                return hip_err(e, "prox_train_step weight and bias gradients");
        } else {
            if (!ok(opf::prox_gemm_mixed(wv, wa, wa_bf16, wlda, h_in, h_in_bf16, fi, gflat + P.wo[k], fi, fo, fi, B,
                                         nullptr, nullptr, false, 0, P.splits[k], skw, s)))
                return hip_err(e, "prox_train_step weight gradient");
            if (!ok(parts ? opf::prox_colsum_parts(cwork, P.chunks, fo, gflat + P.bo[k], 1.0f, s)
                          : opf::prox_colsum(static_cast<const float*>(dpre), B, fo, cwork, gflat + P.bo[k], 1.0f,
                                             s)))
                return hip_err(e, "prox_train_step bias gradient");
        }
        if (k == 0) break;
        const float* pre_below = reinterpret_cast<const float*>(W + P.pre[k - 1]);
        char* d = dbuf[k & 1];
        if (fi % 8 == 0) {
            char* dt = B % 8 == 0 ? dtbuf[k & 1] : nullptr;  // the transposed copy's rows need 16-byte stores
            if (!ok(opf::prox_gemm_gelu_bwd(dpre, d_bf16, fo, weight(k), P.w_bf16[k], fi, pre_below, fi, d, fi, B, fi,
                                            fo, cwork, s, dt, B)))
                return hip_err(e, "prox_train_step dh");
            d_bf16 = parts = true;
            dpreT = dt;
        } else {
            dpreT = nullptr;
            float* dh = reinterpret_cast<float*>(W + P.dh);
            if (!ok(opf::prox_gemm_mixed(1, dpre, d_bf16, fo, weight(k), P.w_bf16[k], fi, dh, fi, B, fi, fo, nullptr,
                                         nullptr, false, 0, 1, nullptr, s)) ||
                !ok(opf::prox_gelu_bwd(pre_below, dh, reinterpret_cast<float*>(d), (int64_t)B * fi, s)))
                return hip_err(e, "prox_train_step dh");
            d_bf16 = parts = false;
        }
        dpre = d;
    }
    pe.mark(3, s);
    if (!ok(opf::prox_adam_dev(mlp->flat, gflat, mlp->m1, mlp->m2, P.n_params, lr, beta1, beta2, eps, mlp->step,
                               mlp->flat_bf16, s)))
        return hip_err(e, "prox_train_step Adam");
    if (phase_ms) {
        pe.mark(4, s);
        if (pe.err != hipSuccess) return hip_err(pe.err, "prox_train_step phase events");
        if (hipError_t r = hipEventSynchronize(pe.ev[4])) return hip_err(r, "prox_train_step phase events");
        for (int i = 0; i < 4; i++)
            if (hipError_t r = hipEventElapsedTime(&phase_ms[i], pe.ev[i], pe.ev[i + 1]))
                return hip_err(r, "prox_train_step phase events");
    }
    return OPF_OK;
}


namespace {
int gemm_checked(int variant, const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb, float* C,
                 int ldc, int M, int N, int K, const float* bias, void* act, bool act_bf16, int accumulate, int splits,
                 float* work, void* stream, const char* what) {
    if (variant < 0 || variant > 3) return set_err(OPF_E_ARG, "variant must be 0..3");
    if (!A || !B) return set_err(OPF_E_ARG, "A and B must be non-NULL");
    if (!C && (!act || accumulate || splits != 1))
        return set_err(OPF_E_ARG, "C may be NULL only with act, no accumulate and one split");
    if (M < 0 || N < 0 || K < 0) return set_err(OPF_E_ARG, "negative dimension");
    if (!mult4(M) || !mult4(N) || !mult4(K) || !mult4(lda) || !mult4(ldb) || !mult4(ldc))
        return set_err(OPF_E_ARG, "dimensions and leading dimensions must be multiples of 4");
    if (!aligned16(A) || !aligned16(B) || (C && !aligned16(C)) || (act && !aligned16(act)))
        return set_err(OPF_E_ARG, "buffers must be 16-byte aligned");
    const bool a_k = variant == 0 || variant == 1, b_k = variant == 0 || variant == 3;
    if (lda < (a_k ? K : M) || ldb < (b_k ? K : N) || ldc < N)
        return set_err(OPF_E_ARG, "a leading dimension is smaller than its row");
    if (((a_bf16 && a_k) || (b_bf16 && b_k)) && (K % 8 || (a_bf16 && a_k && lda % 8) || (b_bf16 && b_k && ldb % 8)))
        return set_err(OPF_E_ARG, "a k-contiguous BF16 operand needs K and its leading dimension multiples of 8");
    if (splits < 1 || splits > 64) return set_err(OPF_E_ARG, "splits must be 1..64");
    if (splits > 1 && (!work || !aligned16(work)))
        return set_err(OPF_E_ARG, "splits > 1 needs a 16-byte aligned work buffer");
    if (M == 0 || N == 0) return OPF_OK;
    return launched(opf::prox_gemm_mixed(variant, A, a_bf16, lda, B, b_bf16, ldb, C, ldc, M, N, K, bias, act, act_bf16,
                                         accumulate, splits, work, static_cast<hipStream_t>(stream)),
                    what);
}
}  // namespace

int prox_gemm_bf16(int variant, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                   int K, const float* bias, float* act, int accumulate, void* stream) {
    return gemm_checked(variant, A, false, lda, B, false, ldb, C, ldc, M, N, K, bias, act, false, accumulate, 1,
                        nullptr, stream, "prox_gemm_bf16 launch");
}

int prox_gemm_bf16_splitk(int variant, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M,
                          int N, int K, const float* bias, float* act, int accumulate, int splits, float* work,
                          void* stream) {
    return gemm_checked(variant, A, false, lda, B, false, ldb, C, ldc, M, N, K, bias, act, false, accumulate, splits,
                        work, stream, "prox_gemm_bf16_splitk launch");
}

int prox_gemm_bf16_mixed(int variant, const void* A, int a_bf16, int lda, const void* B, int b_bf16, int ldb, float* C,
                         int ldc, int M, int N, int K, const float* bias, void* act, int act_bf16, int accumulate,
                         int splits, float* work, void* stream) {
    return gemm_checked(variant, A, a_bf16 != 0, lda, B, b_bf16 != 0, ldb, C, ldc, M, N, K, bias, act, act_bf16 != 0,
                        accumulate, splits, work, stream, "prox_gemm_bf16_mixed launch");
}

int prox_gemm_gelu_bwd(const void* A, int a_bf16, int lda, const void* B, int b_bf16, int ldb, const float* pre,
                       int ldp, void* out, int ldo, int M, int N, int K, float* part, void* stream) {
    if (!A || !B || !pre || !out || !part) return set_err(OPF_E_ARG, "A, B, pre, out and part must be non-NULL");
    if (M < 0 || N < 0 || K < 0) return set_err(OPF_E_ARG, "negative dimension");
    if (!mult4(M) || !mult4(N) || !mult4(K) || !mult4(lda) || !mult4(ldb) || !mult4(ldp) || !mult4(ldo))
        return set_err(OPF_E_ARG, "dimensions and leading dimensions must be multiples of 4");
    if (!aligned16(A) || !aligned16(B) || !aligned16(pre) || (reinterpret_cast<uintptr_t>(out) & 7u))
        return set_err(OPF_E_ARG, "A, B and pre must be 16-byte aligned, out 8-byte aligned");
    if (lda < K || ldb < N || ldp < N || ldo < N) return set_err(OPF_E_ARG, "a leading dimension is smaller than its row");
    if (a_bf16 && (K % 8 || lda % 8))
        return set_err(OPF_E_ARG, "a BF16 A needs K and its leading dimension multiples of 8");
    if (M == 0 || N == 0) return OPF_OK;
    return launched(opf::prox_gemm_gelu_bwd(A, a_bf16 != 0, lda, B, b_bf16 != 0, ldb, pre, ldp, out, ldo, M, N, K,
                                            part, static_cast<hipStream_t>(stream)),
                    "prox_gemm_gelu_bwd launch");
}

int prox_colsum_parts(const float* part, int chunks, int N, float* out, float scale, void* stream) {
    if (chunks < 1 || N < 1 || !part || !out) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_colsum_parts(part, chunks, N, out, scale, static_cast<hipStream_t>(stream)),
                    "prox_colsum_parts launch");
}

int prox_to_bf16(const float* x, int64_t n, void* y, void* stream) {
    if (n < 0 || (n > 0 && (!x || !y))) return set_err(OPF_E_ARG, "bad arguments");
    if (n == 0) return OPF_OK;
    return launched(opf::prox_to_bf16(x, n, y, static_cast<hipStream_t>(stream)), "prox_to_bf16 launch");
}

int prox_gemm_splits(int M, int N, int K) {
    if (M < 0 || N < 0 || K < 0) return set_err(OPF_E_ARG, "negative dimension");
    return opf::prox_gemm_splits(M, N, K);
}

int prox_gelu_bwd(const float* pre, const float* dact, float* dpre, int64_t n, void* stream) {
    if (n < 0 || (n > 0 && (!pre || !dact || !dpre))) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_gelu_bwd(pre, dact, dpre, n, static_cast<hipStream_t>(stream)), "prox_gelu_bwd launch");
}

int prox_colsum(const float* X, int M, int N, float* work, float* out, float scale, void* stream) {
    if (M < 1 || N < 1 || !X || !work || !out) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_colsum(X, M, N, work, out, scale, static_cast<hipStream_t>(stream)), "prox_colsum launch");
}

int prox_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float beta1, float beta2, float eps,
              int step, void* stream) {
    if (n < 0 || step < 1 || (n > 0 && (!p || !g || !m1 || !m2))) return set_err(OPF_E_ARG, "bad arguments");
    if (n == 0) return OPF_OK;
    return launched(opf::prox_adam(p, g, m1, m2, n, lr, beta1, beta2, eps, step, nullptr,
                                   static_cast<hipStream_t>(stream)),
                    "prox_adam launch");
}

int prox_adam_dev(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float beta1, float beta2,
                  float eps, int32_t* step, void* pb, void* stream) {
    if (n < 1 || !p || !g || !m1 || !m2 || !step) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_adam_dev(p, g, m1, m2, n, lr, beta1, beta2, eps, step, pb,
                                       static_cast<hipStream_t>(stream)),
                    "prox_adam_dev launch");
}

int prox_squash_fwd(opf_model model, const float* z, int B, double va_span, double* X, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !z || !X) return set_err(OPF_E_ARG, "bad arguments");
    DeviceGuard dg(model->device);
    return launched(opf::prox_squash_fwd(z, B, box_of(model, va_span), X, model->hm.ly.n, true,
                                         static_cast<hipStream_t>(stream)),
                    "prox_squash_fwd launch");
}

int prox_squash_fwd_vars(opf_model model, const float* z, int B, double va_span, double* X, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !z || !X) return set_err(OPF_E_ARG, "bad arguments");
    DeviceGuard dg(model->device);
    return launched(opf::prox_squash_fwd(z, B, box_of(model, va_span), X, model->hm.ly.n, false,
                                         static_cast<hipStream_t>(stream)),
                    "prox_squash_fwd_vars launch");
}

int prox_squash_bwd(opf_model model, const float* z, int B, double va_span, const double* gX1, const double* gX2,
                    const double* gObj, double obj_scale, float* dz, float scale, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !z || !gX1 || !dz) return set_err(OPF_E_ARG, "bad arguments");
    DeviceGuard dg(model->device);
    return launched(opf::prox_squash_bwd(z, B, box_of(model, va_span), gX1, gX2, gObj, obj_scale, model->hm.ly.n, dz,
                                         (float)scale, static_cast<hipStream_t>(stream)),
                    "prox_squash_bwd launch");
}

int prox_penalty(opf_model model, const double* C, const double* X, const double* F, double obj_scale, double rho,
                 int B, int vjp, double* pen, double* cvio, double* W, double* gpq, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !C || !X || !pen || !cvio || !W) return set_err(OPF_E_ARG, "bad arguments");
    // without gpq the gradient on p, q stays in the workgroup's LDS: only
    // with vjp (its one reader) and when it fits
    constexpr int32_t kMaxOnChip = 7680;  // 60 KiB of doubles beside the 4 KiB of reduction arrays
    if (!gpq && (!vjp || model->hm.ly.L * 4 > kMaxOnChip))
        return set_err(OPF_E_ARG, "gpq may be NULL only with vjp and at most %d arc variables", kMaxOnChip);
    DeviceGuard dg(model->device);
    return launched(opf::prox_penalty(C, X, F, obj_scale, rows_of(model), rho, B, pen, cvio, W, gpq, vjp ? 1 : 0,
                                      static_cast<hipStream_t>(stream)),
                    "prox_penalty launch");
}

int prox_vjp_weights(opf_model model, const double* X, const double* W, const double* gpq, int B, double* Wt,
                     void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !X || !W || !gpq || !Wt) return set_err(OPF_E_ARG, "bad arguments");
    DeviceGuard dg(model->device);
    return launched(opf::prox_vjp_weights(X, W, gpq, rows_of(model), B, Wt, static_cast<hipStream_t>(stream)),
                    "prox_vjp_weights launch");
}

int prox_vjp_sum(opf_model model, const double* X, const double* gX1, const double* gX2, double obj_scale,
                 const double* wb, int B, double* gX, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !gX1 || !wb || !gX) return set_err(OPF_E_ARG, "bad arguments");
    if (obj_scale != 0.0 && !X) return set_err(OPF_E_ARG, "X is needed for the objective term");
    const opf::Layout& ly = model->hm.ly;
    const opf::ProxObj ob{model->dm.c2, model->dm.c1, ly.x_pg, ly.G};
    DeviceGuard dg(model->device);
    return launched(opf::prox_vjp_sum(obj_scale != 0.0 ? X : nullptr, gX1, gX2, ob, obj_scale, wb, B, ly.n, ly.x_p, gX,
                                      static_cast<hipStream_t>(stream)),
                    "prox_vjp_sum launch");
}

int prox_loss_bwd(opf_model model, const float* z, int B, double va_span, const double* X, const double* gX1,
                  double obj_scale, const double* wb, float* dz, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !z || !gX1 || !wb || !dz) return set_err(OPF_E_ARG, "bad arguments");
    if (obj_scale != 0.0 && !X) return set_err(OPF_E_ARG, "X is needed for the objective term");
    const opf::Layout& ly = model->hm.ly;
    const opf::ProxObj ob{model->dm.c2, model->dm.c1, ly.x_pg, ly.G};
    DeviceGuard dg(model->device);
    return launched(opf::prox_loss_bwd(z, B, box_of(model, va_span), ob, obj_scale != 0.0 ? X : nullptr, gX1,
                                       obj_scale, wb, ly.n, dz, static_cast<hipStream_t>(stream)),
                    "prox_loss_bwd launch");
}


int prox_loss_fused_fits(opf_model model) {
    if (!valid_model(model)) return set_err(OPF_E_STATE, "invalid or destroyed model handle");
    return fused_fits(model) ? 1 : 0;
}

int prox_loss_fused(opf_model model, const float* z, int B, double va_span, const double* loads, double rho,
                    double obj_scale, double* loss, double* cvio, double* gz, double* X, double* C, void* stream) {
    if (int rc = static_model(model)) return rc;
    if (B < 1 || !z || !loads || !loss || !cvio) return set_err(OPF_E_ARG, "bad arguments");
    if (!fused_fits(model))
        return set_err(OPF_E_ARG, "the fused loss takes a model without storage or devices whose sample fits "
                                  "%zu bytes of LDS",
                       kFusedLdsMax);
    DeviceGuard dg(model->device);
    const opf::ProxPerm pm{model->he_pos, model->gen_pos};
    return launched(opf::prox_loss_fused(model->dm, box_of(model, va_span), rows_of(model), pm, z, loads, B, rho,
                                         obj_scale, loss, cvio, gz, X, C, static_cast<hipStream_t>(stream)),
                    "prox_loss_fused launch");
}

int prox_sample_loads(const double* r, const double* base, const double* inv_scale, double spread, int B, int N,
                      double* loads, float* feats, void* stream) {
    if (B < 1 || N < 1 || !r || !base || !inv_scale || !loads || !feats) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_sample_loads(r, base, inv_scale, spread, B, N, loads, feats,
                                           static_cast<hipStream_t>(stream)),
                    "prox_sample_loads launch");
}

int prox_scale_rows(const double* gz, const double* wb, int B, int D, float* dz, void* stream) {
    if (B < 1 || D < 1 || !gz || !wb || !dz) return set_err(OPF_E_ARG, "bad arguments");
    return launched(opf::prox_scale_rows(gz, wb, 0.0, B, D, dz, static_cast<hipStream_t>(stream)),
                    "prox_scale_rows launch");
}

}  // extern "C"
