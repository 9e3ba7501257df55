// gfx950 kernels of the learned warm-start proxy: a multilayer perceptron
// that maps bus loads to (vm, va, pg, qg), trained with a penalty on the
// FP64 constraint violation that the callback kernels compute.
//
//  - prox_gemm: C[M,N] = A[M,K] B[K,N] on the matrix cores
//    (v_mfma_f32_32x32x16_bf16): operands are FP32 in memory, rounded to
//    BF16 (nearest even) when staged into LDS, accumulated in FP32; optional
//    fused epilogue bias + exact GELU.  128x128 block tile, BK = 32, four
//    waves of 64x64, global loads of the next K tile overlapped with the
//    matrix-core work on the current one.
//  - elementwise / reduction kernels: GELU backward, deterministic column
//    sums (bias gradient), Adam, output squashing into the variable bounds
//    and its backward, the penalty loss with its constraint weights, and the
//    chain weights that carry the arc-flow gradient back to the voltages.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "proxy_kernels.h"

namespace opf {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK + 8;  // LDS row stride (bf16) with padding against bank conflicts
constexpr int GEMM_THREADS = 256;

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    // d/dx x Phi(x) = Phi(x) + x phi(x)
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Loads one BM x BK tile of A (rows i, columns k) or one BN x BK tile of B^T
// (rows j, columns k) as 16 floats per thread, zero outside the matrix.
// KCONT: k is the contiguous memory index (row stride ld); otherwise the row
// index is contiguous (k stride ld).
template <bool KCONT>
__device__ __forceinline__ void load_tile(const float* __restrict__ P, int ld, int rows, int K, int r0, int k0,
                                          float4 (&reg)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        int r, k;
        if (KCONT) {
            r = r0 + t / 8 + 32 * q;
            k = k0 + (t % 8) * 4;
        } else {
            k = k0 + t / 32 + 8 * q;
            r = r0 + (t % 32) * 4;
        }
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (KCONT) {
            if (r < rows && k < K) v = *reinterpret_cast<const float4*>(P + (size_t)r * ld + k);
        } else {
            if (k < K && r < rows) v = *reinterpret_cast<const float4*>(P + (size_t)k * ld + r);
        }
        reg[q] = v;
    }
}

template <bool KCONT>
__device__ __forceinline__ void store_tile(__bf16* S, const float4 (&reg)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float4 v = reg[q];
        if (KCONT) {
            const int r = t / 8 + 32 * q, k = (t % 8) * 4;
            __bf16* d = S + r * LDK + k;
            d[0] = to_bf16(v.x);
            d[1] = to_bf16(v.y);
            d[2] = to_bf16(v.z);
            d[3] = to_bf16(v.w);
        } else {
            const int k = t / 32 + 8 * q, r = (t % 32) * 4;
            S[(r + 0) * LDK + k] = to_bf16(v.x);
            S[(r + 1) * LDK + k] = to_bf16(v.y);
            S[(r + 2) * LDK + k] = to_bf16(v.z);
            S[(r + 3) * LDK + k] = to_bf16(v.w);
        }
    }
}

// C[M,N] = A[M,K] B[K,N] (+ bias[N], then optionally GELU into act).
//  A_KCONT: A(i,k) = A[i*lda + k], else A[k*lda + i]
//  B_KCONT: B(k,j) = B[j*ldb + k], else B[k*ldb + j]
template <bool A_KCONT, bool B_KCONT>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_kernel(const float* __restrict__ A, int lda,
                                                            const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                            int ldc, int M, int N, int K,
                                                            const float* __restrict__ bias, float* __restrict__ act,
                                                            int accumulate) {
    __shared__ __bf16 As[BM * LDK];
    __shared__ __bf16 Bs[BN * LDK];
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wi = (wave / 2) * 64, wj = (wave % 2) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[a][b][v] = 0.f;

    float4 ra[4], rb[4];
    load_tile<A_KCONT>(A, lda, M, K, i0, 0, ra);
    load_tile<B_KCONT>(B, ldb, N, K, j0, 0, rb);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store_tile<A_KCONT>(As, ra);
        store_tile<B_KCONT>(Bs, rb);
        __syncthreads();
        if (k0 + BK < K) {  // next tile's global loads overlap the matrix-core work
            load_tile<A_KCONT>(A, lda, M, K, i0, k0 + BK, ra);
            load_tile<B_KCONT>(B, ldb, N, K, j0, k0 + BK, rb);
        }
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int kk = ks + (lane / 32) * 8;
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; a++)
                fa[a] = *reinterpret_cast<const bf16x8*>(As + (wi + a * 32 + lane % 32) * LDK + kk);
#pragma unroll
            for (int b = 0; b < 2; b++)
                fb[b] = *reinterpret_cast<const bf16x8*>(Bs + (wj + b * 32 + lane % 32) * LDK + kk);
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
    }
    // epilogue: lane holds column j = lane % 32 of each 32x32 tile, rows
    // (v / 4) * 8 + (lane / 32) * 4 + v % 4
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int j = j0 + wj + b * 32 + lane % 32;
            if (j >= N) continue;
            const float bj = bias ? bias[j] : 0.f;
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int i = i0 + wi + a * 32 + (v / 4) * 8 + (lane / 32) * 4 + v % 4;
                if (i >= M) continue;
                float r = acc[a][b][v] + bj;
                float* cp = C + (size_t)i * ldc + j;
                if (accumulate) r += *cp;
                *cp = r;
                if (act) act[(size_t)i * ldc + j] = gelu(r);
            }
        }
}

__global__ void gelu_bwd_kernel(const float* __restrict__ pre, const float* __restrict__ dact,
                                float* __restrict__ dpre, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dpre[i] = dact[i] * gelu_grad(pre[i]);
}

// Column sums of a row-major [M, N] matrix, deterministic: partial sums over
// fixed 256-row chunks, then the chunks in order.
constexpr int COLSUM_ROWS = 256;
__global__ void colsum_partial_kernel(const float* __restrict__ X, int M, int N, float* __restrict__ part) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= N) return;
    const int i0 = c * COLSUM_ROWS, i1 = min(i0 + COLSUM_ROWS, M);
    float s = 0.f;
    for (int i = i0; i < i1; i++) s += X[(size_t)i * N + j];
    part[(size_t)c * N + j] = s;
}
__global__ void colsum_final_kernel(const float* __restrict__ part, int chunks, int N, float* __restrict__ out,
                                    float scale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int c = 0; c < chunks; c++) s += part[(size_t)c * N + j];
    out[j] = s * scale;
}

// Adam (Kingma and Ba, 2015) with bias correction; FP32 state.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__device__ __forceinline__ double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

// z [B, 2N + 2G] (vm, va, pg, qg blocks, FP32) -> the first 2N + 2G entries
// of each instance's x [B, n] (va, vm, pg, qg, FP64); p and q are zeroed.
__global__ void squash_fwd_kernel(const float* __restrict__ z, int B, ProxBox box, double* __restrict__ X,
                                  int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = box.N, G = box.G;
    const int64_t per = n;
    if (idx >= (int64_t)B * per) return;
    const int64_t b = idx / per;
    const int64_t e = idx % per;
    const float* zb = z + b * (2 * (int64_t)N + 2 * G);
    double v;
    if (e < N) {  // va
        v = box.is_ref[e] ? 0.0 : box.va_span * tanh((double)zb[N + e]);
    } else if (e < 2 * N) {  // vm
        const int i = (int)(e - N);
        v = box.vmin[i] + (box.vmax[i] - box.vmin[i]) * sigmoid((double)zb[i]);
    } else if (e < 2 * N + G) {
        const int k = (int)(e - 2 * N);
        v = box.pmin[k] + (box.pmax[k] - box.pmin[k]) * sigmoid((double)zb[2 * N + k]);
    } else if (e < 2 * N + 2 * G) {
        const int k = (int)(e - 2 * N - G);
        v = box.qmin[k] + (box.qmax[k] - box.qmin[k]) * sigmoid((double)zb[2 * N + G + k]);
    } else {
        v = 0.0;
    }
    X[idx] = v;
}

// dz from dL/dx = gX + gX2 + obj_scale * gObj on the (va, vm, pg, qg)
// entries (gX2, gObj may be NULL).
__global__ void squash_bwd_kernel(const float* __restrict__ z, int B, ProxBox box, const double* __restrict__ gX1,
                                  const double* __restrict__ gX2, const double* __restrict__ gObj, double obj_scale,
                                  int64_t n, float* __restrict__ dz, float scale) {
    const int D = 2 * box.N + 2 * box.G;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * D) return;
    const int64_t b = idx / D;
    const int j = (int)(idx % D);
    const int N = box.N, G = box.G;
    const double zj = z[idx];
    // the x entry this output feeds
    int64_t e;
    if (j < N) e = N + j;                    // vm
    else if (j < 2 * N) e = j - N;           // va
    else e = j;                              // pg, qg: same offset in z and x
    double g = gX1[b * n + e];
    if (gX2) g += gX2[b * n + e];
    if (gObj) g += obj_scale * gObj[b * n + e];
    double d;
    if (j < N) {  // vm
        const double s = sigmoid(zj);
        d = g * (box.vmax[j] - box.vmin[j]) * s * (1.0 - s);
    } else if (j < 2 * N) {  // va
        const int i = j - N;
        const double t = tanh(zj);
        d = box.is_ref[i] ? 0.0 : g * box.va_span * (1.0 - t * t);
    } else if (j < 2 * N + G) {
        const int k = j - 2 * N;
        const double s = sigmoid(zj);
        d = g * (box.pmax[k] - box.pmin[k]) * s * (1.0 - s);
    } else {
        const int k = j - 2 * N - G;
        const double s = sigmoid(zj);
        d = g * (box.qmax[k] - box.qmin[k]) * s * (1.0 - s);
    }
    dz[idx] = (float)(d * scale);
}

// Per instance b: the loss rho * (sum over non-flow rows of viol^2 + sum
// over p, q of bound viol^2) + obj_scale * F[b] (F may be NULL), the
// constraint violation (max over all rows and variable bounds), the weights
// w = d penalty / d c (zero on flow rows) and d penalty / d x on the p, q
// entries.  One workgroup per instance, fixed-order reduction.
__global__ void __launch_bounds__(256) penalty_kernel(const double* __restrict__ C, const double* __restrict__ X,
                                                      const double* __restrict__ F, double obj_scale,
                                                      ProxRows rows, double rho, double* __restrict__ pen,
                                                      double* __restrict__ cvio, double* __restrict__ W,
                                                      double* __restrict__ gpq) {
    __shared__ double s_pen[256], s_vio[256];
    const int64_t b = blockIdx.x;
    const double* c = C + b * rows.m;
    const double* x = X + b * rows.n;
    double* w = W + b * rows.m;
    double* gq = gpq + b * rows.npq;
    double sp = 0.0, sv = 0.0;
    for (int r = threadIdx.x; r < rows.m; r += 256) {
        const double cr = c[r];
        const double lo = rows.lcon[r], hi = rows.ucon[r];
        const double dv = cr < lo ? cr - lo : (cr > hi ? cr - hi : 0.0);
        sv = fmax(sv, fabs(dv));
        const bool flow = r >= rows.flow0 && r < rows.flow1;
        if (!flow) sp += dv * dv;
        w[r] = flow ? 0.0 : 2.0 * rho * dv;
    }
    for (int q = threadIdx.x; q < rows.npq; q += 256) {
        const double xv = x[rows.pq0 + q];
        const double lo = rows.lvar[rows.pq0 + q], hi = rows.uvar[rows.pq0 + q];
        const double dv = xv < lo ? xv - lo : (xv > hi ? xv - hi : 0.0);
        sv = fmax(sv, fabs(dv));
        sp += dv * dv;
        gq[q] = 2.0 * rho * dv;
    }
    s_pen[threadIdx.x] = sp;
    s_vio[threadIdx.x] = sv;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s_pen[threadIdx.x] += s_pen[threadIdx.x + s];
            s_vio[threadIdx.x] = fmax(s_vio[threadIdx.x], s_vio[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pen[b] = F ? rho * s_pen[0] + obj_scale * F[b] : rho * s_pen[0];
        cvio[b] = s_vio[0];
    }
}

// The arc flows p, q are F(vm, va); a gradient g on them reaches the voltages
// through the flow rows c = p - F: J^T w2 with w2 = -g on the flow rows
// carries -dF^T (-g) = dF^T g to va, vm.  Writes w2 (zero off the flow rows).
__global__ void chain_weights_kernel(const double* __restrict__ G1, const double* __restrict__ gpq, ProxRows rows,
                                     int B, double* __restrict__ W2) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * rows.m) return;
    const int64_t b = idx / rows.m;
    const int r = (int)(idx % rows.m);
    double w = 0.0;
    if (r >= rows.flow0 && r < rows.flow1) {
        // flow rows: p_fr[L], q_fr[L], p_to[L], q_to[L]; arc variable of each
        const int L = rows.L;
        const int rr = r - rows.flow0;
        const int blk = rr / L, l = rr % L;
        const int arc = (blk == 0 || blk == 1) ? l : L + l;
        const int isq = (blk == 1 || blk == 3);
        const int q = isq * 2 * L + arc;  // index inside the p, q entries
        w = -(G1[b * rows.n + rows.pq0 + q] + gpq[b * rows.npq + q]);
    }
    W2[idx] = w;
}

// gX [B, n] = wb[b] * (gX1 + gX2 + obj_scale * gObj) on the va, vm, pg, qg
// entries (the free variables of the proxy), zero on the arc variables.
__global__ void vjp_sum_kernel(const double* __restrict__ gX1, const double* __restrict__ gX2,
                               const double* __restrict__ gObj, double obj_scale, const double* __restrict__ wb,
                               int B, int64_t n, int64_t nfree, double* __restrict__ gX) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * n) return;
    const int64_t b = idx / n, e = idx % n;
    double g = 0.0;
    if (e < nfree) {
        g = gX1[idx];
        if (gX2) g += gX2[idx];
        if (gObj) g += obj_scale * gObj[idx];
        g *= wb[b];
    }
    gX[idx] = g;
}

}  // namespace

hipError_t prox_vjp_sum(const double* gX1, const double* gX2, const double* gObj, double obj_scale,
                        const double* wb, int B, int64_t n, int64_t nfree, double* gX, hipStream_t s) {
    const int64_t tot = (int64_t)B * n;
    hipLaunchKernelGGL(vjp_sum_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, gX1, gX2, gObj,
                       obj_scale, wb, B, n, nfree, gX);
    return hipGetLastError();
}

hipError_t prox_gemm(int variant, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                     int K, const float* bias, float* act, int accumulate, hipStream_t s) {
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM), block(GEMM_THREADS);
    switch (variant) {
    case 0: hipLaunchKernelGGL((gemm_kernel<true, true>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, bias, act, accumulate); break;
    case 1: hipLaunchKernelGGL((gemm_kernel<true, false>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, bias, act, accumulate); break;
    case 2: hipLaunchKernelGGL((gemm_kernel<false, false>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, bias, act, accumulate); break;
    default: hipLaunchKernelGGL((gemm_kernel<false, true>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, bias, act, accumulate); break;
    }
    return hipGetLastError();
}

hipError_t prox_gelu_bwd(const float* pre, const float* dact, float* dpre, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gelu_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pre, dact, dpre, n);
    return hipGetLastError();
}

hipError_t prox_colsum(const float* X, int M, int N, float* part, float* out, float scale, hipStream_t s) {
    const int chunks = (M + COLSUM_ROWS - 1) / COLSUM_ROWS;
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((N + 255) / 256, chunks), dim3(256), 0, s, X, M, N, part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0, s, part, chunks, N, out, scale);
    return hipGetLastError();
}

int prox_colsum_chunks(int M) { return (M + COLSUM_ROWS - 1) / COLSUM_ROWS; }

hipError_t prox_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                     int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m1, m2, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t prox_squash_fwd(const float* z, int B, const ProxBox& box, double* X, int64_t n, hipStream_t s) {
    const int64_t tot = (int64_t)B * n;
    hipLaunchKernelGGL(squash_fwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, B, box, X, n);
    return hipGetLastError();
}

hipError_t prox_squash_bwd(const float* z, int B, const ProxBox& box, const double* gX1, const double* gX2,
                           const double* gObj, double obj_scale, int64_t n, float* dz, float scale, hipStream_t s) {
    const int64_t tot = (int64_t)B * (2 * box.N + 2 * box.G);
    hipLaunchKernelGGL(squash_bwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, B, box, gX1, gX2,
                       gObj, obj_scale, n, dz, scale);
    return hipGetLastError();
}

hipError_t prox_penalty(const double* C, const double* X, const double* F, double obj_scale, const ProxRows& rows,
                        double rho, int B, double* pen, double* cvio, double* W, double* gpq, hipStream_t s) {
    hipLaunchKernelGGL(penalty_kernel, dim3(B), dim3(256), 0, s, C, X, F, obj_scale, rows, rho, pen, cvio, W, gpq);
    return hipGetLastError();
}

hipError_t prox_chain_weights(const double* G1, const double* gpq, const ProxRows& rows, int B, double* W2,
                              hipStream_t s) {
    const int64_t tot = (int64_t)B * rows.m;
    hipLaunchKernelGGL(chain_weights_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, G1, gpq, rows, B,
                       W2);
    return hipGetLastError();
}

}  // namespace opf
