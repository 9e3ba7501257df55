// Launchers of the warm-start proxy kernels (proxy_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace opf {

struct DevModel;

// Variable boxes of one model (device pointers) for the output squashing.
struct ProxBox {
    int32_t N, G;
    const double *vmin, *vmax, *pmin, *pmax, *qmin, *qmax;
    const int32_t* is_ref;  // [N] 1 for a reference bus (its angle stays 0)
    double va_span;         // va = va_span * tanh(z)
};

// Constraint rows and bounds of one model (device pointers) for the penalty.
struct ProxRows {
    int32_t m, n, L;
    int32_t flow0, flow1;   // the flow-definition rows [flow0, flow1)
    int32_t pq0, npq;       // the p and q variables [pq0, pq0 + npq)
    int32_t thf, tht;       // first rows of the from / to thermal blocks
    int32_t balp, balq;     // first rows of the active / reactive balance blocks
    const double *lcon, *ucon, *lvar, *uvar;
    const int32_t *f_bus, *t_bus;  // branch end buses
};

// variant: 0 A k-contiguous, B k-contiguous; 1 A k-contiguous, B j-contiguous;
//          2 A i-contiguous, B j-contiguous; 3 A i-contiguous, B k-contiguous.
// splits > 1: the k range in that many parts into work (splits * M * N
// floats), then summed in order with the epilogue.
hipError_t prox_gemm(int variant, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                     int K, const float* bias, float* act, int accumulate, int splits, float* work, hipStream_t s);
// prox_gemm with either operand stored as BF16 (a_bf16, b_bf16) and the GELU
// output stored as BF16 (act_bf16); a k-contiguous BF16 operand has K and its
// leading dimension multiples of 8.
hipError_t prox_gemm_mixed(int variant, const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                           float* C, int ldc, int M, int N, int K, const float* bias, void* act, bool act_bf16,
                           int accumulate, int splits, float* work, hipStream_t s);
int prox_gemm_splits(int M, int N, int K);
// The split-K parts only (splits >= 2) of prox_gemm_mixed without bias,
// activation or accumulation: work receives splits * M * N floats.
hipError_t prox_gemm_split_parts(int variant, const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                                 int M, int N, int K, int splits, float* work, hipStream_t s);
// C [M, N] = the split-K parts summed in order, and bias_out [NB] = the
// column sums of part [chunks, NB] (prox_colsum's second pass), one launch.
hipError_t prox_wgrad_finish(const float* work, int splits, int M, int N, float* C, int ldc, const float* part,
                             int chunks, int NB, float* bias_out, hipStream_t s);
// out [M, N] (BF16) = (A B) * gelu'(pre) for row-major A [M, K], B [K, N]
// (either BF16), pre [M, N]; part [ceil(M / 128), N] = the column sums of
// each 128-row block of the FP32 product (prox_colsum's first pass); outT
// (optional) = out transposed, [N, M] with leading dimension ldT (a
// multiple of 8, outT 16-byte aligned).
hipError_t prox_gemm_gelu_bwd(const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                              const float* pre, int ldp, void* out, int ldo, int M, int N, int K, float* part,
                              hipStream_t s, void* outT = nullptr, int ldT = 0);
// out [N] = scale * the column sums of part [chunks, N] (prox_colsum's second pass)
hipError_t prox_colsum_parts(const float* part, int chunks, int N, float* out, float scale, hipStream_t s);
hipError_t prox_gelu_bwd(const float* pre, const float* dact, float* dpre, int64_t n, hipStream_t s);
hipError_t prox_colsum(const float* X, int M, int N, float* part, float* out, float scale, hipStream_t s);
// prox_colsum's first pass only: part [ceil(M / 128), N]
hipError_t prox_colsum_first(const float* X, int M, int N, float* part, hipStream_t s);
hipError_t prox_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                     int step, void* pb, hipStream_t s);
hipError_t prox_adam_dev(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                         float eps, int32_t* step, void* pb, hipStream_t s);
hipError_t prox_to_bf16(const float* x, int64_t n, void* y, hipStream_t s);
// arcs: also set the arc variables p, q to 0 (else they are left as they are)
hipError_t prox_squash_fwd(const float* z, int B, const ProxBox& box, double* X, int64_t n, bool arcs, hipStream_t s);
hipError_t prox_squash_bwd(const float* z, int B, const ProxBox& box, const double* gX1, const double* gX2,
                           const double* gObj, double obj_scale, int64_t n, float* dz, float scale, hipStream_t s);
hipError_t prox_penalty(const double* C, const double* X, const double* F, double obj_scale, const ProxRows& rows,
                        double rho, int B, double* pen, double* cvio, double* W, double* gpq, int vjp, hipStream_t s);
hipError_t prox_vjp_weights(const double* X, const double* W, const double* gpq, const ProxRows& rows, int B,
                            double* Wt, hipStream_t s);
// The objective's cost coefficients (device) and pg block of a static model.
struct ProxObj {
    const double *c2, *c1;
    int64_t x_pg, G;
};
hipError_t prox_vjp_sum(const double* X, const double* gX1, const double* gX2, const ProxObj& ob, double obj_scale,
                        const double* wb, int B, int64_t n, int64_t nfree, double* gX, hipStream_t s);
hipError_t prox_loss_bwd(const float* z, int B, const ProxBox& box, const ProxObj& ob, const double* X,
                         const double* gX1, double obj_scale, const double* wb, int64_t n, float* dz, hipStream_t s);

// The fused FP64 loss of B samples of one static polar model (one
// workgroup each, the sample's working set in prox_loss_fused_lds bytes of
// LDS): loss, cvio [B]; gz [B, 2N+2G] = d loss_b / d z_b (NULL: not
// computed); X [B, n], C [B, m] on request (NULL: not written).  loads [B, 2N]
// holds each sample's pd then qd.
struct ProxPerm {
    const int32_t* he_pos;   // [2L] position of (side, branch) in the bus-ordered half-edge list, from sides first
    const int32_t* gen_pos;  // [G] position of generator k in the bus-ordered generator list
};
size_t prox_loss_fused_lds(int N, int L, int G);
// dz (optional, in place of gz) = (float)(w * d loss_b / d z_b).
hipError_t prox_loss_fused(const DevModel& m, const ProxBox& box, const ProxRows& rows, const ProxPerm& pm,
                           const float* z, const double* loads, int B, double rho, double obj_scale, double* loss,
                           double* cvio, double* gz, double* X, double* C, hipStream_t s, float* dz = nullptr,
                           double w = 0.0);
// loads [B, 2N] and FP32 features [B, 2N] of the proxy's samples from
// uniform draws r [B, N] (prox_sample_loads)
hipError_t prox_sample_loads(const double* r, const double* base, const double* inv_scale, double spread, int B,
                             int N, double* loads, float* feats, hipStream_t s);
// dz [B, D] = (float)(w_b * gz[b, j]), w_b = wb[b] or, with wb NULL, w
hipError_t prox_scale_rows(const double* gz, const double* wb, double w, int B, int D, float* dz, hipStream_t s);

}  // namespace opf
