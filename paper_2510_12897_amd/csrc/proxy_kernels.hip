// gfx950 kernels of the learned warm-start proxy: a multilayer perceptron
// that maps bus loads to (vm, va, pg, qg), trained with a penalty on the
// FP64 constraint violation that the callback kernels compute.
//
//  - prox_gemm / prox_gemm_mixed: C[M,N] = A[M,K] B[K,N] on the matrix
//    cores (v_mfma_f32_32x32x16_bf16), FP32 accumulation: each operand is
//    either FP32 in memory, rounded to BF16 (nearest even) when staged into
//    LDS, or already BF16 (the MLP's weight copy and hidden activations);
//    optional fused epilogue bias + exact GELU (FP32 or BF16 output), staged
//    through LDS for whole-row vector stores.  128x128 or 128x64 block tile,
//    BK = 64, four waves of 64x64 or 64x32, global loads of the next K tile
//    overlapped with the matrix-core work on the current one.
//  - prox_gemm_gelu_bwd: the dh product with the GELU backward of the layer
//    below and the bias gradient's first column-sum pass in its epilogue.
//  - the fused loss (prox_loss_fused): the whole FP64 side of a sample in one
//    workgroup's LDS (squashing, arc flows, rows, penalty, Cvio, d loss / d z).
//  - elementwise / reduction kernels: GELU backward, deterministic column
//    sums (bias gradient), Adam (also with its step count on the device and
//    a BF16 copy of the parameters, 16-byte accesses where aligned), the
//    samples' loads and features, output squashing into the variable
//    bounds and its backward (also fused with the objective and loss-weight
//    step), the penalty loss with its constraint weights, and the chain
//    weights that carry the arc-flow gradient back to the voltages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dev_model.h"
#include "proxy_kernels.h"

namespace opf {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int BM = 128, BK = 64;  // block tile rows (of A / C) and k depth; columns: 128 or 64
constexpr int GEMM_THREADS = 256;
constexpr int kXcd = 8;       // accelerator complex dies, each with its own L2
constexpr int kWideMin = 512; // 128-column tiles only when they give two workgroups per CU (256 CUs)

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    // d/dx x Phi(x) = Phi(x) + x phi(x)
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// LDS operand tile: 128 rows (i of A, j of B) of BK = 64 BF16 values, eight
// 16-byte chunks of 8 k values per row.  Chunk c of row r sits at position
// c ^ ((r >> 1) & 7): the fragment reads (16 consecutive rows, one chunk) and
// the row-wise tile stores then fall on distinct banks.
__device__ __forceinline__ int lds_at(int r, int c) { return r * BK + ((c ^ ((r >> 1) & 7)) << 3); }

__device__ __forceinline__ bf16x8 pack8(float a0, float a1, float a2, float a3, float a4, float a5, float a6,
                                        float a7) {
    return (bf16x8){to_bf16(a0), to_bf16(a1), to_bf16(a2), to_bf16(a3),
                    to_bf16(a4), to_bf16(a5), to_bf16(a6), to_bf16(a7)};
}

// Global loads of one ROWS x BK operand tile (rows r0.., k0..; ROWS = 128 or
// 64), ROWS / 8 floats per thread, zero outside rows < nrows, k < kend.
// Sizes are multiples of 4, so each float4 is wholly inside or outside.
//  KCONT: element (r, k) at P[r * ld + k]; thread t holds row t / 8 + 32 q,
//         k = 8 (t % 8) .. + 8 as v[2q], v[2q + 1].
//  else:  element (r, k) at P[k * ld + r]; thread t holds the four rows
//         4 (t % G) .. + 4 (G = ROWS / 4 row groups) at the k values
//         K (t / G) + kk, K = 4 G / 8 (8 for 128 rows, 4 for 64), as v[kk]:
//         a coalesced row segment per k.
__device__ __forceinline__ float4 guarded_load(const float* __restrict__ base, const float* p, bool ok) {
    // an out-of-range load reads the (valid) first element and is discarded
    const float4 t = *reinterpret_cast<const float4*>(ok ? p : base);
    return ok ? t : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Registers that stage one operand tile between its global load and its LDS
// store: FP32 operands as float4 (rounded to BF16 at the store); BF16
// operands as they are stored (k-contiguous: 8 k values of one row per
// 16-byte load; i-contiguous: 4 rows of one k per 8-byte load).
template <typename T, bool KCONT, int ROWS>
struct TileRegs {
    float4 v[ROWS / 16];
};
template <int ROWS>
struct TileRegs<__bf16, true, ROWS> {
    uint4 v[ROWS / 32];
};
template <int ROWS>
struct TileRegs<__bf16, false, ROWS> {
    uint2 v[ROWS / 16];
};

template <bool KCONT, int ROWS>
__device__ __forceinline__ void load_tile(const float* __restrict__ P, int ld, int nrows, int kend, int r0, int k0,
                                          TileRegs<float, KCONT, ROWS>& R) {
    float4 (&v)[ROWS / 16] = R.v;
    const int t = threadIdx.x;
    if (KCONT) {
        const int k = k0 + (t % 8) * 8;
#pragma unroll
        for (int q = 0; q < ROWS / 32; q++) {
            const int r = r0 + t / 8 + 32 * q;
            const float* p = P + (size_t)r * ld + k;
            v[2 * q] = guarded_load(P, p, r < nrows && k < kend);
            v[2 * q + 1] = guarded_load(P, p + 4, r < nrows && k + 4 < kend);
        }
    } else {
        constexpr int G = ROWS / 4, KPER = ROWS / 16;
        const int r = r0 + (t % G) * 4;
#pragma unroll
        for (int kk = 0; kk < KPER; kk++) {
            const int k = k0 + (t / G) * KPER + kk;
            v[kk] = guarded_load(P, P + (size_t)k * ld + r, r < nrows && k < kend);
        }
    }
}

// Rounds the loaded tile to BF16 and writes it to LDS as row chunks (the
// i-contiguous layout is transposed in registers: 16-byte chunks for 128
// rows, 8-byte half chunks for 64).
template <bool KCONT, int ROWS>
__device__ __forceinline__ void store_tile(__bf16* S, const TileRegs<float, KCONT, ROWS>& R) {
    const float4 (&v)[ROWS / 16] = R.v;
    const int t = threadIdx.x;
    if (KCONT) {
#pragma unroll
        for (int q = 0; q < ROWS / 32; q++) {
            const float4 a = v[2 * q], b = v[2 * q + 1];
            *reinterpret_cast<bf16x8*>(S + lds_at(t / 8 + 32 * q, t % 8)) =
                pack8(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
        }
    } else if (ROWS == 128) {
        const int r = (t % 32) * 4, c = t / 32;
        *reinterpret_cast<bf16x8*>(S + lds_at(r + 0, c)) =
            pack8(v[0].x, v[1].x, v[2].x, v[3].x, v[4].x, v[5].x, v[6].x, v[7].x);
        *reinterpret_cast<bf16x8*>(S + lds_at(r + 1, c)) =
            pack8(v[0].y, v[1].y, v[2].y, v[3].y, v[4].y, v[5].y, v[6].y, v[7].y);
        *reinterpret_cast<bf16x8*>(S + lds_at(r + 2, c)) =
            pack8(v[0].z, v[1].z, v[2].z, v[3].z, v[4].z, v[5].z, v[6].z, v[7].z);
        *reinterpret_cast<bf16x8*>(S + lds_at(r + 3, c)) =
            pack8(v[0].w, v[1].w, v[2].w, v[3].w, v[4].w, v[5].w, v[6].w, v[7].w);
    } else {
        const int r = (t % 16) * 4, kq = t / 16;  // k = 4 kq .. + 4: half kq % 2 of chunk kq / 2
        const int c = kq / 2, h = (kq % 2) * 4;
        *reinterpret_cast<bf16x4*>(S + lds_at(r + 0, c) + h) =
            (bf16x4){to_bf16(v[0].x), to_bf16(v[1].x), to_bf16(v[2].x), to_bf16(v[3].x)};
        *reinterpret_cast<bf16x4*>(S + lds_at(r + 1, c) + h) =
            (bf16x4){to_bf16(v[0].y), to_bf16(v[1].y), to_bf16(v[2].y), to_bf16(v[3].y)};
        *reinterpret_cast<bf16x4*>(S + lds_at(r + 2, c) + h) =
            (bf16x4){to_bf16(v[0].z), to_bf16(v[1].z), to_bf16(v[2].z), to_bf16(v[3].z)};
        *reinterpret_cast<bf16x4*>(S + lds_at(r + 3, c) + h) =
            (bf16x4){to_bf16(v[0].w), to_bf16(v[1].w), to_bf16(v[2].w), to_bf16(v[3].w)};
    }
}

// BF16 operands: the same thread-to-element maps as the FP32 loads above.
// A k-contiguous operand has its k extent and leading dimension multiples
// of 8, so that every 16-byte load of 8 k values is wholly inside or outside.
template <bool KCONT, int ROWS>
__device__ __forceinline__ void load_tile(const __bf16* __restrict__ P, int ld, int nrows, int kend, int r0, int k0,
                                          TileRegs<__bf16, KCONT, ROWS>& R) {
    const int t = threadIdx.x;
    if constexpr (KCONT) {
        const int k = k0 + (t % 8) * 8;
#pragma unroll
        for (int q = 0; q < ROWS / 32; q++) {
            const int r = r0 + t / 8 + 32 * q;
            const bool ok = r < nrows && k < kend;
            const uint4 u = *reinterpret_cast<const uint4*>(ok ? P + (size_t)r * ld + k : P);
            R.v[q] = ok ? u : make_uint4(0u, 0u, 0u, 0u);
        }
    } else {
        constexpr int G = ROWS / 4, KPER = ROWS / 16;
        const int r = r0 + (t % G) * 4;
#pragma unroll
        for (int kk = 0; kk < KPER; kk++) {
            const int k = k0 + (t / G) * KPER + kk;
            const bool ok = r < nrows && k < kend;
            const uint2 u = *reinterpret_cast<const uint2*>(ok ? P + (size_t)k * ld + r : P);
            R.v[kk] = ok ? u : make_uint2(0u, 0u);
        }
    }
}

__device__ __forceinline__ uint32_t pack_lo(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
__device__ __forceinline__ uint32_t pack_hi(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

template <bool KCONT, int ROWS>
__device__ __forceinline__ void store_tile(__bf16* S, const TileRegs<__bf16, KCONT, ROWS>& R) {
    const int t = threadIdx.x;
    if constexpr (KCONT) {
#pragma unroll
        for (int q = 0; q < ROWS / 32; q++) *reinterpret_cast<uint4*>(S + lds_at(t / 8 + 32 * q, t % 8)) = R.v[q];
    } else if constexpr (ROWS == 128) {
        // thread: rows r .. r + 3 at k values 8 c .. 8 c + 7 (v[kk] = rows at k = 8 c + kk)
        const uint2* v = R.v;
        const int r = (t % 32) * 4, c = t / 32;
        *reinterpret_cast<uint4*>(S + lds_at(r + 0, c)) =
            make_uint4(pack_lo(v[0].x, v[1].x), pack_lo(v[2].x, v[3].x), pack_lo(v[4].x, v[5].x), pack_lo(v[6].x, v[7].x));
        *reinterpret_cast<uint4*>(S + lds_at(r + 1, c)) =
            make_uint4(pack_hi(v[0].x, v[1].x), pack_hi(v[2].x, v[3].x), pack_hi(v[4].x, v[5].x), pack_hi(v[6].x, v[7].x));
        *reinterpret_cast<uint4*>(S + lds_at(r + 2, c)) =
            make_uint4(pack_lo(v[0].y, v[1].y), pack_lo(v[2].y, v[3].y), pack_lo(v[4].y, v[5].y), pack_lo(v[6].y, v[7].y));
        *reinterpret_cast<uint4*>(S + lds_at(r + 3, c)) =
            make_uint4(pack_hi(v[0].y, v[1].y), pack_hi(v[2].y, v[3].y), pack_hi(v[4].y, v[5].y), pack_hi(v[6].y, v[7].y));
    } else {
        const uint2* v = R.v;
        const int r = (t % 16) * 4, kq = t / 16;  // k = 4 kq .. + 4: half kq % 2 of chunk kq / 2
        const int c = kq / 2, h = (kq % 2) * 4;
        *reinterpret_cast<uint2*>(S + lds_at(r + 0, c) + h) = make_uint2(pack_lo(v[0].x, v[1].x), pack_lo(v[2].x, v[3].x));
        *reinterpret_cast<uint2*>(S + lds_at(r + 1, c) + h) = make_uint2(pack_hi(v[0].x, v[1].x), pack_hi(v[2].x, v[3].x));
        *reinterpret_cast<uint2*>(S + lds_at(r + 2, c) + h) = make_uint2(pack_lo(v[0].y, v[1].y), pack_lo(v[2].y, v[3].y));
        *reinterpret_cast<uint2*>(S + lds_at(r + 3, c) + h) = make_uint2(pack_hi(v[0].y, v[1].y), pack_hi(v[2].y, v[3].y));
    }
}

// One BK-deep step of a wave's 64 x (32 NB) tile from the LDS operands.
template <int NB>
__device__ __forceinline__ void mma_tile(const __bf16* As, const __bf16* Bs, int wi, int wj, int lane,
                                         f32x16 (&acc)[2][NB]) {
#pragma unroll
    for (int ks = 0; ks < BK / 16; ks++) {
        const int c = ks * 2 + lane / 32;
        bf16x8 fa[2], fb[NB];
#pragma unroll
        for (int a = 0; a < 2; a++)
            fa[a] = *reinterpret_cast<const bf16x8*>(As + lds_at(wi + a * 32 + lane % 32, c));
#pragma unroll
        for (int b = 0; b < NB; b++)
            fb[b] = *reinterpret_cast<const bf16x8*>(Bs + lds_at(wj + b * 32 + lane % 32, c));
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < NB; b++)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
}

// C[M,N] = A[M,K] B[K,N] (+ bias[N], then optionally GELU into act).
//  A_KCONT: A(i,k) = A[i*lda + k], else A[k*lda + i]
//  B_KCONT: B(k,j) = B[j*ldb + k], else B[k*ldb + j]
// A workgroup computes one 128 x BN tile (BN = 128 or 64) over the k range
// [z kchunk, (z + 1) kchunk); with work != NULL it writes that partial product
// to work[z] (row-major [M, N]) instead of the epilogue.  Four waves of 64 x 64,
// double-buffered LDS (one barrier per k tile), the next tile's global loads
// in flight during the matrix-core work on the current one.
// TA, TB: the operands' storage (float, rounded when staged, or __bf16);
// TACT: the storage of the GELU output.
// The operand tiles in LDS, and after the k loop the epilogue's staging tile.
template <int BN>
constexpr int gemm_smem_bytes() {
    return (2 * BM * BK + 2 * BN * BK) * (int)sizeof(__bf16);
}

// The k loop of one output tile: the XCD-aware tile of this workgroup
// (i0, j0, k part kz) and its accumulators.  Workgroups are dealt to the
// XCDs round-robin; they are renumbered so that each XCD takes one
// contiguous range of tiles (n fastest, then m, then the k part): its rows of
// A and the shared B stay in its own L2.
template <bool A_KCONT, bool B_KCONT, int BN, typename TA, typename TB>
__device__ __forceinline__ void gemm_mainloop(const TA* __restrict__ A, int lda, const TB* __restrict__ B, int ldb,
                                              int M, int N, int K, int kchunk, char* smem, int& i0, int& j0, int& kz,
                                              f32x16 (&acc)[2][BN / 64]) {
    constexpr int NB = BN / 64;  // 32-column MFMA tiles per wave
    __bf16 (*As)[BM * BK] = reinterpret_cast<__bf16 (*)[BM * BK]>(smem);
    __bf16 (*Bs)[BN * BK] = reinterpret_cast<__bf16 (*)[BN * BK]>(smem + 2 * BM * BK * sizeof(__bf16));
    const int nx = gridDim.x, ny = gridDim.y, nb = nx * ny * gridDim.z;
    const int bl = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const int q = nb / kXcd, rem = nb % kXcd, xcd = bl % kXcd;
    const int tile = xcd * q + min(xcd, rem) + bl / kXcd;
    i0 = (tile / nx) % ny * BM;
    j0 = tile % nx * BN;
    kz = tile / (nx * ny);
    const int kb = kz * kchunk, ke = min(K, kb + kchunk);
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wi = (wave / 2) * 64, wj = (wave % 2) * (BN / 2);
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[a][b][v] = 0.f;

    TileRegs<TA, A_KCONT, BM> ra;
    TileRegs<TB, B_KCONT, BN> rb;
    if (kb < ke) {
        load_tile<A_KCONT, BM>(A, lda, M, ke, i0, kb, ra);
        load_tile<B_KCONT, BN>(B, ldb, N, ke, j0, kb, rb);
        store_tile<A_KCONT, BM>(As[0], ra);
        store_tile<B_KCONT, BN>(Bs[0], rb);
    }
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += BK) {
        const bool more = k0 + BK < ke;
        if (more) {
            load_tile<A_KCONT, BM>(A, lda, M, ke, i0, k0 + BK, ra);
            load_tile<B_KCONT, BN>(B, ldb, N, ke, j0, k0 + BK, rb);
        }
        mma_tile<NB>(As[cur], Bs[cur], wi, wj, lane, acc);
        if (more) {  // the other buffer: every wave passed the last barrier after reading it
            store_tile<A_KCONT, BM>(As[cur ^ 1], ra);
            store_tile<B_KCONT, BN>(Bs[cur ^ 1], rb);
        }
        __syncthreads();
        cur ^= 1;
    }
}

template <bool A_KCONT, bool B_KCONT, int BN, typename TA, typename TB, typename TACT>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_kernel(const TA* __restrict__ A, int lda,
                                                            const TB* __restrict__ B, int ldb, float* __restrict__ C,
                                                            int ldc, int M, int N, int K, int kchunk,
                                                            const float* __restrict__ bias, TACT* __restrict__ act,
                                                            int accumulate, float* __restrict__ work) {
    constexpr int NB = BN / 64;  // 32-column MFMA tiles per wave
    __shared__ __align__(16) char smem[gemm_smem_bytes<BN>()];
    int i0, j0, kz;
    f32x16 acc[2][NB];
    gemm_mainloop<A_KCONT, B_KCONT, BN>(A, lda, B, ldb, M, N, K, kchunk, smem, i0, j0, kz, acc);
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wi = (wave / 2) * 64, wj = (wave % 2) * (BN / 2);
    // Lane holds column lane % 32 of each 32x32 tile, rows (v / 4) * 8 +
    // (lane / 32) * 4 + v % 4.
    // Epilogue through LDS, in two halves of 64 rows: the a = 0 (then
    // a = 1) accumulator tiles of every wave go to a row-major staging tile,
    // then each thread takes 4 consecutive columns of a row and stores them
    // as one 16-byte C vector (and one act vector), so that a wave writes
    // whole rows instead of 4-byte values (forward 4096 x 1024 x 1024: 27.6
    // -> 24.8 us).  The last k-loop barrier freed the operand tiles.
    if (work) {  // a split-K part: the raw partial product, stored directly (measured faster than staged)
        float* W = work + (size_t)kz * M * N;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int j = j0 + wj + b * 32 + lane % 32;
                if (j >= N) continue;
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int i = i0 + wi + a * 32 + (v / 4) * 8 + (lane / 32) * 4 + v % 4;
                    if (i < M) W[(size_t)i * N + j] = acc[a][b][v];
                }
            }
        return;
    }
    constexpr int SROW = BN + 4;  // padded row stride of the staging tile (floats)
    constexpr int C4 = BN / 4;    // 4-column groups per row
    float* stage = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int a = 0; a < 2; a++) {
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int lr = (wave / 2) * 32 + (v / 4) * 8 + (lane / 32) * 4 + v % 4;
                stage[lr * SROW + wj + b * 32 + lane % 32] = acc[a][b][v];
            }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * C4; e += GEMM_THREADS) {
            const int lr = e / C4, c4 = e % C4;
            const int i = i0 + (lr / 32) * 64 + a * 32 + lr % 32;  // staging row -> output row
            const int j = j0 + c4 * 4;
            if (i >= M || j >= N) continue;
            float4 r = *reinterpret_cast<const float4*>(stage + lr * SROW + c4 * 4);
            if (bias) {
                r.x += bias[j];
                r.y += bias[j + 1];
                r.z += bias[j + 2];
                r.w += bias[j + 3];
            }
            if (C) {  // NULL: act is the only output (the host allows it without accumulate)
                float4* cp = reinterpret_cast<float4*>(C + (size_t)i * ldc + j);
                if (accumulate) {
                    const float4 c0 = *cp;
                    r.x += c0.x;
                    r.y += c0.y;
                    r.z += c0.z;
                    r.w += c0.w;
                }
                *cp = r;
            }
            if (act) {
                TACT* ap = act + (size_t)i * ldc + j;
                if constexpr (sizeof(TACT) == 2)
                    *reinterpret_cast<bf16x4*>(ap) = (bf16x4){to_bf16(gelu(r.x)), to_bf16(gelu(r.y)),
                                                              to_bf16(gelu(r.z)), to_bf16(gelu(r.w))};
                else
                    *reinterpret_cast<float4*>(ap) = make_float4(gelu(r.x), gelu(r.y), gelu(r.z), gelu(r.w));
            }
        }
        __syncthreads();
    }
}

// dgrad with the GELU backward of the layer below in the epilogue (64-column
// tiles): d = (A B) * gelu'(pre), stored as BF16 (the operand rounding every
// later product applies anyway), and the column sums of each 128-row block of
// d in FP32 (the bias gradient's first pass), summed in the order of
// colsum_partial_kernel (rows g, g + 4, ... for g = 0..3, then the four
// groups in order), so the values equal the GEMM, gelu_bwd and colsum
// kernels in sequence bit for bit.
// outT (may be NULL) receives d transposed, [N, M] BF16 with leading
// dimension ldT (a multiple of 8): the k-contiguous operand of the next
// weight-gradient product.
template <bool A_KCONT, bool B_KCONT, typename TA, typename TB>
__global__ void __launch_bounds__(GEMM_THREADS) gemm_gelu_bwd_kernel(const TA* __restrict__ A, int lda,
                                                                     const TB* __restrict__ B, int ldb,
                                                                     const float* __restrict__ pre, int ldp,
                                                                     __bf16* __restrict__ out, int ldo, int M, int N,
                                                                     int K, float* __restrict__ part,
                                                                     __bf16* __restrict__ outT, int ldT) {
    constexpr int BN = 64, SROW = BN + 4, C4 = BN / 4;
    // the whole 128 x 64 FP32 tile (padded rows) and the column-sum groups fit the operand tiles' LDS
    static_assert(BM * SROW * 4 + 4 * 64 * 4 <= gemm_smem_bytes<BN>(), "staging tile");
    __shared__ __align__(16) char smem[gemm_smem_bytes<BN>()];
    int i0, j0, kz;
    f32x16 acc[2][1];
    gemm_mainloop<A_KCONT, B_KCONT, BN>(A, lda, B, ldb, M, N, K, K, smem, i0, j0, kz, acc);
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wi = (wave / 2) * 64, wj = (wave % 2) * (BN / 2);
    float* stage = reinterpret_cast<float*>(smem);
    float (*sg)[64] = reinterpret_cast<float (*)[64]>(smem + BM * SROW * 4);
    // Lane holds column lane % 32 of each 32x32 tile, rows (v / 4) * 8 +
    // (lane / 32) * 4 + v % 4; the last k-loop barrier freed the operand tiles.
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int v = 0; v < 16; v++)
            stage[(wi + a * 32 + (v / 4) * 8 + (lane / 32) * 4 + v % 4) * SROW + wj + lane % 32] = acc[a][0][v];
    __syncthreads();
    for (int e = threadIdx.x; e < BM * C4; e += GEMM_THREADS) {
        const int lr = e / C4, c4 = e % C4;
        const int i = i0 + lr, j = j0 + c4 * 4;
        if (i >= M || j >= N) continue;
        float4* sp = reinterpret_cast<float4*>(stage + lr * SROW + c4 * 4);
        const float4 dh = *sp;
        const float4 pr = *reinterpret_cast<const float4*>(pre + (size_t)i * ldp + j);
        const float4 d = make_float4(dh.x * gelu_grad(pr.x), dh.y * gelu_grad(pr.y), dh.z * gelu_grad(pr.z),
                                     dh.w * gelu_grad(pr.w));
        *reinterpret_cast<bf16x4*>(out + (size_t)i * ldo + j) =
            (bf16x4){to_bf16(d.x), to_bf16(d.y), to_bf16(d.z), to_bf16(d.w)};
        *sp = d;
    }
    __syncthreads();
    const int c = threadIdx.x % 64, g = threadIdx.x / 64, j = j0 + c;
    const int rows = min(BM, M - i0);
    if (outT && j < N) {  // 8 consecutive rows of column j per 16-byte store
        __bf16* tcol = outT + (size_t)j * ldT + i0;
        for (int r0 = g * 8; r0 < rows; r0 += 32) {
            if (r0 + 8 <= rows) {
                bf16x8 v;
#pragma unroll
                for (int q = 0; q < 8; q++) v[q] = to_bf16(stage[(r0 + q) * SROW + c]);
                *reinterpret_cast<bf16x8*>(tcol + r0) = v;
            } else {
                for (int q = r0; q < rows; q++) tcol[q] = to_bf16(stage[q * SROW + c]);
            }
        }
    }
    float s = 0.f;
    if (j < N)
        for (int r = g; r < rows; r += 4) s += stage[r * SROW + c];
    sg[g][c] = s;
    __syncthreads();
    if (g == 0 && j < N) part[(size_t)(i0 / BM) * N + j] = ((sg[0][c] + sg[1][c]) + sg[2][c]) + sg[3][c];
}

// Split-K epilogue: C = sum over the parts in order (part 0 first) + bias
// (+ C when accumulating), GELU into act; four columns per thread.
template <typename TACT>
__global__ void splitk_sum_kernel(const float* __restrict__ work, int splits, int M, int N, float* __restrict__ C,
                                  int ldc, const float* __restrict__ bias, TACT* __restrict__ act, int accumulate) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n4 = N / 4;
    if (idx >= (int64_t)M * n4) return;
    const int i = (int)(idx / n4), j = (int)(idx % n4) * 4;
    const size_t mn = (size_t)M * N;
    const float* w = work + (size_t)i * N + j;
    float4 s = *reinterpret_cast<const float4*>(w);
    for (int z = 1; z < splits; z++) {
        const float4 t = *reinterpret_cast<const float4*>(w + z * mn);
        s.x += t.x;
        s.y += t.y;
        s.z += t.z;
        s.w += t.w;
    }
    if (bias) {
        s.x += bias[j];
        s.y += bias[j + 1];
        s.z += bias[j + 2];
        s.w += bias[j + 3];
    }
    float4* cp = reinterpret_cast<float4*>(C + (size_t)i * ldc + j);
    if (accumulate) {
        const float4 c = *cp;
        s.x += c.x;
        s.y += c.y;
        s.z += c.z;
        s.w += c.w;
    }
    *cp = s;
    if (act) {
        TACT* ap = act + (size_t)i * ldc + j;
        ap[0] = (TACT)gelu(s.x);
        ap[1] = (TACT)gelu(s.y);
        ap[2] = (TACT)gelu(s.z);
        ap[3] = (TACT)gelu(s.w);
    }
}

__global__ void gelu_bwd_kernel(const float* __restrict__ pre, const float* __restrict__ dact,
                                float* __restrict__ dpre, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dpre[i] = dact[i] * gelu_grad(pre[i]);
}

// Column sums of a row-major [M, N] matrix, deterministic.  Pass 1: per
// 128-row chunk and 64-column stripe, four row groups (rows g, g + 4, ...)
// each sum in row order, then the four groups in order.  Pass 2: the chunk
// sums of each column the same way (chunks g, g + 4, ..., then the groups).
constexpr int COLSUM_ROWS = 128;
__global__ void __launch_bounds__(256) colsum_partial_kernel(const float* __restrict__ X, int M, int N,
                                                             float* __restrict__ part) {
    __shared__ float s[4][64];
    const int c = threadIdx.x % 64, g = threadIdx.x / 64;
    const int j = blockIdx.x * 64 + c;
    const int i0 = blockIdx.y * COLSUM_ROWS, i1 = min(i0 + COLSUM_ROWS, M);
    float acc = 0.f;
    if (j < N)
        for (int i = i0 + g; i < i1; i += 4) acc += X[(size_t)i * N + j];
    s[g][c] = acc;
    __syncthreads();
    if (g == 0 && j < N) part[(size_t)blockIdx.y * N + j] = ((s[0][c] + s[1][c]) + s[2][c]) + s[3][c];
}
__global__ void __launch_bounds__(256) colsum_final_kernel(const float* __restrict__ part, int chunks, int N,
                                                           float* __restrict__ out, float scale) {
    __shared__ float s[4][64];
    const int c = threadIdx.x % 64, g = threadIdx.x / 64;
    const int j = blockIdx.x * 64 + c;
    float acc = 0.f;
    if (j < N)
        for (int k = g; k < chunks; k += 4) acc += part[(size_t)k * N + j];
    s[g][c] = acc;
    __syncthreads();
    if (g == 0 && j < N) out[j] = (((s[0][c] + s[1][c]) + s[2][c]) + s[3][c]) * scale;
}

// The end of a weight gradient in one launch: blocks [0, nsum) sum the
// split-K parts into C [M, N] in part order (splitk_sum_kernel without
// epilogue); the remaining blocks do the bias gradient's second column-sum
// pass over part [chunks, NB] (colsum_final_kernel, scale 1).  The same
// values as those two kernels, one launch fewer.
__global__ void __launch_bounds__(256) wgrad_finish_kernel(const float* __restrict__ work, int splits, int M, int N,
                                                           float* __restrict__ C, int ldc, int nsum,
                                                           const float* __restrict__ part, int chunks, int NB,
                                                           float* __restrict__ bias_out) {
    if ((int)blockIdx.x < nsum) {
        const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const int n4 = N / 4;
        if (idx >= (int64_t)M * n4) return;
        const int i = (int)(idx / n4), j = (int)(idx % n4) * 4;
        const size_t mn = (size_t)M * N;
        const float* w = work + (size_t)i * N + j;
        float4 sv = *reinterpret_cast<const float4*>(w);
        for (int z = 1; z < splits; z++) {
            const float4 t = *reinterpret_cast<const float4*>(w + z * mn);
            sv.x += t.x;
            sv.y += t.y;
            sv.z += t.z;
            sv.w += t.w;
        }
        *reinterpret_cast<float4*>(C + (size_t)i * ldc + j) = sv;
        return;
    }
    __shared__ float sg[4][64];
    const int c = threadIdx.x % 64, g = threadIdx.x / 64;
    const int j = ((int)blockIdx.x - nsum) * 64 + c;
    float acc = 0.f;
    if (j < NB)
        for (int k = g; k < chunks; k += 4) acc += part[(size_t)k * NB + j];
    sg[g][c] = acc;
    __syncthreads();
    if (g == 0 && j < NB) bias_out[j] = (((sg[0][c] + sg[1][c]) + sg[2][c]) + sg[3][c]) * 1.0f;
}

// Adam (Kingma and Ba, 2015) with bias correction; FP32 state.
// pb (may be NULL) receives the updated parameters rounded to BF16: the
// matrix cores' copy of the weights.
// One parameter's Adam update (Kingma and Ba, Algorithm 1, with the bias
// corrections c1, c2).  No contraction, so that every kernel below rounds
// each operation alike whatever the compiler would fuse in its context.
__device__ __forceinline__ void adam_one(float& p, float g, float& m1, float& m2, float lr, float b1, float b2,
                                         float eps, float c1, float c2) {
#pragma clang fp contract(off)
    const float a = b1 * m1 + (1.f - b1) * g;
    const float b = b2 * m2 + (1.f - b2) * g * g;
    m1 = a;
    m2 = b;
    p = p - lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2, __bf16* __restrict__ pb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float pi = p[i], ai = m1[i], bi = m2[i];
    adam_one(pi, g[i], ai, bi, lr, b1, b2, eps, c1, c2);
    m1[i] = ai;
    m2[i] = bi;
    p[i] = pi;
    if (pb) pb[i] = to_bf16(pi);
}

// Adam with the step count in device memory (a recorded step replays with
// the count it finds there): each workgroup forms the bias corrections from
// step + 1, and step_bump_kernel, launched after it, stores step + 1.
__global__ void adam_dev_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                                float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps,
                                const int32_t* __restrict__ step, __bf16* __restrict__ pb) {
    __shared__ float corr[2];  // the bias corrections, formed once per workgroup
    if (threadIdx.x == 0) {
        const float t = (float)(*step + 1);
        corr[0] = 1.f - powf(b1, t);
        corr[1] = 1.f - powf(b2, t);
    }
    __syncthreads();
    const float c1 = corr[0], c2 = corr[1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float pi = p[i], ai = m1[i], bi = m2[i];
    adam_one(pi, g[i], ai, bi, lr, b1, b2, eps, c1, c2);
    m1[i] = ai;
    m2[i] = bi;
    p[i] = pi;
    if (pb) pb[i] = to_bf16(pi);
}

// adam_dev_kernel over 4 consecutive parameters per thread (16-byte
// accesses) in a grid-stride loop: the same arithmetic per parameter, the
// bias corrections formed once per workgroup for many more parameters.
__global__ void __launch_bounds__(256) adam_dev4_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                        float* __restrict__ m1, float* __restrict__ m2, int64_t n,
                                                        float lr, float b1, float b2, float eps,
                                                        const int32_t* __restrict__ step, __bf16* __restrict__ pb) {
    __shared__ float corr[2];
    if (threadIdx.x == 0) {
        const float t = (float)(*step + 1);
        corr[0] = 1.f - powf(b1, t);
        corr[1] = 1.f - powf(b2, t);
    }
    __syncthreads();
    const float c1 = corr[0], c2 = corr[1];
    const int64_t n4 = n / 4, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
        float4 pv = reinterpret_cast<float4*>(p)[q];
        float4 av = reinterpret_cast<float4*>(m1)[q];
        float4 bv = reinterpret_cast<float4*>(m2)[q];
        const float4 gv = reinterpret_cast<const float4*>(g)[q];
        adam_one(pv.x, gv.x, av.x, bv.x, lr, b1, b2, eps, c1, c2);
        adam_one(pv.y, gv.y, av.y, bv.y, lr, b1, b2, eps, c1, c2);
        adam_one(pv.z, gv.z, av.z, bv.z, lr, b1, b2, eps, c1, c2);
        adam_one(pv.w, gv.w, av.w, bv.w, lr, b1, b2, eps, c1, c2);
        reinterpret_cast<float4*>(m1)[q] = av;
        reinterpret_cast<float4*>(m2)[q] = bv;
        reinterpret_cast<float4*>(p)[q] = pv;
        if (pb)
            reinterpret_cast<bf16x4*>(pb)[q] = (bf16x4){to_bf16(pv.x), to_bf16(pv.y), to_bf16(pv.z), to_bf16(pv.w)};
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float pi = p[i], ai = m1[i], bi = m2[i];
        adam_one(pi, g[i], ai, bi, lr, b1, b2, eps, c1, c2);
        m1[i] = ai;
        m2[i] = bi;
        p[i] = pi;
        if (pb) pb[i] = to_bf16(pi);
    }
}

__global__ void step_bump_kernel(int32_t* step) { *step += 1; }

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, __bf16* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

__device__ __forceinline__ double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

// Entry e < 2N + 2G (va, vm, pg, qg blocks of x) of the squashed network
// output zb (vm, va, pg, qg blocks, FP32), and in act the activation it
// came from (tanh for va, the sigmoid otherwise): the squashing kernel and
// the fused loss kernel both call it, so both write the same bits.
__device__ __forceinline__ double squash_entry(const ProxBox& box, const float* zb, int e, double& act) {
    const int N = box.N, G = box.G;
    if (e < N) {  // va
        act = tanh((double)zb[N + e]);
        return box.is_ref[e] ? 0.0 : box.va_span * act;
    }
    if (e < 2 * N) {  // vm
        const int i = e - N;
        act = sigmoid((double)zb[i]);
        return box.vmin[i] + (box.vmax[i] - box.vmin[i]) * act;
    }
    if (e < 2 * N + G) {
        const int k = e - 2 * N;
        act = sigmoid((double)zb[2 * N + k]);
        return box.pmin[k] + (box.pmax[k] - box.pmin[k]) * act;
    }
    const int k = e - 2 * N - G;
    act = sigmoid((double)zb[2 * N + G + k]);
    return box.qmin[k] + (box.qmax[k] - box.qmin[k]) * act;
}

// z [B, 2N + 2G] (vm, va, pg, qg blocks, FP32) -> the first 2N + 2G entries
// of each instance's x [B, n] (va, vm, pg, qg, FP64); p and q are zeroed.
// per = n writes every entry (p, q = 0); per = 2N + 2G leaves p, q as they are.
__global__ void squash_fwd_kernel(const float* __restrict__ z, int B, ProxBox box, double* __restrict__ X,
                                  int64_t n, int64_t per) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int D = 2 * box.N + 2 * box.G;
    if (idx >= (int64_t)B * per) return;
    const int64_t b = idx / per;
    const int64_t e = idx % per;
    double act;
    X[b * n + e] = e < D ? squash_entry(box, z + b * D, (int)e, act) : 0.0;
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

// dz = (d x / d z)^T g with g = wb[b] (gX1 + obj_scale grad f(X)) on the
// va, vm, pg, qg entries (grad f = 2 c2 pg + c1 on pg): the objective and
// loss-weight step of vjp_sum_kernel and squash_bwd_kernel in one pass, in
// the same order of operations.
__global__ void loss_bwd_kernel(const float* __restrict__ z, int B, ProxBox box, ProxObj ob,
                                const double* __restrict__ X, const double* __restrict__ gX1, double obj_scale,
                                const double* __restrict__ wb, int64_t n, float* __restrict__ dz) {
    const int D = 2 * box.N + 2 * box.G;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * D) return;
    const int64_t b = idx / D;
    const int j = (int)(idx % D);
    const int N = box.N, G = box.G;
    const double zj = z[idx];
    int64_t e;
    if (j < N) e = N + j;                    // vm
    else if (j < 2 * N) e = j - N;           // va
    else e = j;                              // pg, qg: same offset in z and x
    double g = gX1[b * n + e];
    if (X && j >= 2 * N && j < 2 * N + G) {
        const int k = j - 2 * N;
        g += obj_scale * (2.0 * ob.c2[k] * X[b * n + e] + ob.c1[k]);
    }
    g *= wb[b];
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
    dz[idx] = (float)d;
}

// The arc flows p, q are F(vm, va): a gradient on them reaches the
// voltages through the flow rows c = p - F, whose va / vm columns are -dF.
// With G1 = J^T W, the arc entry of the total gradient is G1 + gpq, and
// J^T W2 with w2 = -(G1 + gpq) on the arc's flow row carries it to va, vm.
// G1 has a closed form on the arc variables: column p_a of J holds the flow
// row (weight 0 in W), the branch side's thermal row (2 p_a) and the active
// balance row of the arc's bus (1); q_a likewise with the reactive row.  So
// the total weights Wt = W + W2 need no first product, and the VJP is the
// single product J^T Wt.  w2 of flow row rr (0 .. 4L) of one instance:
__device__ __forceinline__ double flow_weight(const double* x, const double* w, const double* gq, const ProxRows& rows,
                                              int rr) {
    // flow rows p_fr[L], q_fr[L], p_to[L], q_to[L]
    const int L = rows.L;
    const int blk = rr / L, l = rr % L;
    const bool from = blk == 0 || blk == 1, isq = blk == 1 || blk == 3;
    const int q = (isq ? 2 * L : 0) + (from ? l : L + l);  // index inside the p, q entries
    const int bus = from ? rows.f_bus[l] : rows.t_bus[l];
    const double g1 = 2.0 * x[rows.pq0 + q] * w[(from ? rows.thf : rows.tht) + l] + w[(isq ? rows.balq : rows.balp) + bus];
    return -(g1 + gq[q]);
}

// Per instance b: the loss rho * (sum over non-flow rows of viol^2 + sum
// over p, q of bound viol^2) + obj_scale * F[b] (F may be NULL), the
// constraint violation (max over all rows and variable bounds), the weights
// w = d penalty / d c (zero on flow rows) and d penalty / d x on the p, q
// entries.  One workgroup per instance, fixed-order reduction.
__global__ void __launch_bounds__(256) penalty_kernel(const double* __restrict__ C, const double* __restrict__ X,
                                                      const double* __restrict__ F, double obj_scale,
                                                      ProxRows rows, double rho, double* __restrict__ pen,
                                                      double* __restrict__ cvio, double* W, double* gpq, int vjp) {
    __shared__ double s_pen[256], s_vio[256];
    extern __shared__ double s_gq[];  // d pen / d (p, q) when gpq is NULL (vjp only)
    const int64_t b = blockIdx.x;
    const double* c = C + b * rows.m;
    const double* x = X + b * rows.n;
    double* w = W + b * rows.m;
    double* gq = gpq ? gpq + b * rows.npq : s_gq;
    double sp = 0.0, sv = 0.0;
    for (int r = threadIdx.x; r < rows.m; r += 256) {
        const double cr = c[r];
        const double lo = rows.lcon[r], hi = rows.ucon[r];
        const double dv = cr < lo ? cr - lo : (cr > hi ? cr - hi : 0.0);
        sv = fmax(sv, fabs(dv));
        const bool flow = r >= rows.flow0 && r < rows.flow1;
        if (!flow) sp += dv * dv;
        if (!(flow && vjp)) w[r] = flow ? 0.0 : 2.0 * rho * dv;  // with vjp the flow rows come below
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
    if (vjp) {  // the workgroup's W and gpq stores are visible after the barriers above
        for (int rr = threadIdx.x; rr < rows.flow1 - rows.flow0; rr += 256)
            w[rows.flow0 + rr] = flow_weight(x, w, gq, rows, rr);
    }
}

// The VJP weights on their own (prox_vjp_weights): one thread per flow row.
// The flow rows of Wt are written from W's thermal and balance rows, which
// they never overlap, so Wt may be W itself; a separate Wt also receives W's
// other rows.
__global__ void vjp_weights_kernel(const double* X, const double* W, const double* __restrict__ gpq, ProxRows rows,
                                   int B, double* Wt) {
    const int nf = rows.flow1 - rows.flow0;  // 4 L
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * nf) return;
    const int64_t b = idx / nf;
    const int rr = (int)(idx % nf);
    Wt[b * rows.m + rows.flow0 + rr] = flow_weight(X + b * rows.n, W + b * rows.m, gpq + b * rows.npq, rows, rr);
}
__global__ void copy_off_flow_kernel(const double* __restrict__ W, ProxRows rows, int B, double* __restrict__ Wt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * rows.m) return;
    const int r = (int)(idx % rows.m);
    if (r < rows.flow0 || r >= rows.flow1) Wt[idx] = W[idx];
}

// gX [B, n] = wb[b] * (gX1 + gX2 + obj_scale * grad f) on the va, vm, pg, qg
// entries (the free variables of the proxy), zero on the arc variables;
// grad f = 2 c2 pg + c1 on the pg entries, 0 elsewhere (static model).
__global__ void vjp_sum_kernel(const double* __restrict__ X, const double* __restrict__ gX1,
                               const double* __restrict__ gX2, ProxObj ob, double obj_scale,
                               const double* __restrict__ wb, int B, int64_t n, int64_t nfree,
                               double* __restrict__ gX) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * n) return;
    const int64_t b = idx / n, e = idx % n;
    double g = 0.0;
    if (e < nfree) {
        g = gX1[idx];
        if (gX2) g += gX2[idx];
        if (X && e >= ob.x_pg && e < ob.x_pg + ob.G) {
            const int64_t k = e - ob.x_pg;
            g += obj_scale * (2.0 * ob.c2[k] * X[idx] + ob.c1[k]);
        }
        g *= wb[b];
    }
    gX[idx] = g;
}

// The proxy's training samples from uniform draws r [B, N] in [0, 1): bus
// i's pd and qd both scaled by 1 + spread (2 r - 1); loads [B, 2N] (pd then
// qd) and the network's features (loads - base) * inv_scale as FP32.  The
// operations of the host formula one by one, uncontracted.
__global__ void sample_loads_kernel(const double* __restrict__ r, const double* __restrict__ base,
                                    const double* __restrict__ inv_scale, double spread, int B, int N,
                                    double* __restrict__ loads, float* __restrict__ feats) {
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)B * 2 * N;
    if (idx >= tot) return;
    const int64_t b = idx / (2 * N);
    const int j = (int)(idx % (2 * N)), i = j < N ? j : j - N;
    const double u = r[b * N + i] * 2.0 - 1.0;
    const double fac = 1.0 + spread * u;
    const double l = base[j] * fac;
    loads[idx] = l;
    feats[idx] = (float)((l - base[j]) * inv_scale[j]);
}

// ------------------------------------------------------------ fused loss
// The whole FP64 side of the training loss in one launch, one workgroup per
// sample, every intermediate in LDS: squashing, the arc flows p, q := F(vm,
// va), the non-flow rows (reference, angle, balance, thermal), the penalty,
// the largest violation and, when asked, d loss / d z.  Only z, the loads
// and the model's read-only arrays are read, and only the loss, Cvio and
// d loss / d z are written (X and C on request): about 14 KB per 300-bus
// sample, where the chain of batch launches moves [B, n] and [B, m] arrays
// through HBM several times.
//
// The gradient is the same chain as the penalty VJP (J^T of the row
// weights, carried to the voltages through the flows), written per branch
// and summed per bus over the bus's half-edges in adjacency order (no
// atomics: the same bits on every run).
//
// Flow, thermal-row and objective-term arithmetic is not contracted, as in
// the callback kernels, so the arc flows, thermal rows and X equal those of
// the batch launches bit for bit; the per-bus and per-sample sums are
// ordered differently (rounding-level differences in the balance rows, the
// loss and the gradient).
constexpr int kFuseThreads = 256;

// F = al u^2 + be w^2 + u w (a C + b S) and its derivatives in u, w and the
// angle difference (the expression of the callback kernels' flow terms).
struct PFlow {
    double F, Fu, Fw, Ft;
};
__device__ __forceinline__ PFlow pflow(double al, double be, double a, double b, double u, double w, double C,
                                       double S) {
#pragma clang fp contract(off)
    const double k1 = a * C + b * S;
    const double k2 = b * C - a * S;
    const double uw = u * w;
    PFlow r;
    r.F = al * u * u + be * w * w + uw * k1;
    r.Fu = 2.0 * al * u + w * k1;
    r.Fw = 2.0 * be * w + u * k1;
    r.Ft = uw * k2;
    return r;
}

__device__ __forceinline__ double viol(double v, double lo, double hi) {
    return v < lo ? v - lo : (v > hi ? v - hi : 0.0);
}

__device__ __forceinline__ double wave_sum64(double v) {
    for (int s = 32; s > 0; s >>= 1) v += __shfl_down(v, s, 64);
    return v;
}
__device__ __forceinline__ double wave_max64(double v) {
    for (int s = 32; s > 0; s >>= 1) v = fmax(v, __shfl_down(v, s, 64));
    return v;
}

// The four flows of branch l at the voltages in LDS: p_f, q_f, p_t, q_t,
// with cos and sin of the angle difference in C, S (computed here when
// TRIG, else taken as given).
struct BranchFlows {
    PFlow pf, qf, pt, qt;
    int fb, tb;
};
template <bool TRIG>
__device__ __forceinline__ BranchFlows branch_flows(const DevModel& m, int l, const double* s_va, const double* s_vm,
                                                    double& C, double& S) {
    const int L = m.L;
    BranchFlows r;
    r.fb = m.f_bus[l];
    r.tb = m.t_bus[l];
    const double* k = m.coef + l;  // Gff Bff Gft Bft Gtt Btt Gtf Btf, L apart
    const double Gff = k[0], Bff = k[L], Gft = k[2 * L], Bft = k[3 * L];
    const double Gtt = k[4 * L], Btt = k[5 * L], Gtf = k[6 * L], Btf = k[7 * L];
    const double u = s_vm[r.fb], w = s_vm[r.tb];
    if (TRIG) sincos(s_va[r.fb] - s_va[r.tb], &S, &C);
    r.pf = pflow(Gff, 0.0, Gft, Bft, u, w, C, S);
    r.qf = pflow(-Bff, 0.0, -Bft, Gft, u, w, C, S);
    r.pt = pflow(0.0, Gtt, Gtf, -Btf, u, w, C, S);
    r.qt = pflow(0.0, -Btt, -Btf, -Gtf, u, w, C, S);
    return r;
}

// What one branch contributes to the penalty, from its arc values in LDS
// (half-edge positions hf, ht): the thermal, angle and arc-bound
// violations.  A pass over the branches in two loops, the flows first (with
// the trigonometry) and then this, holds fewer registers than one loop
// doing both, so more workgroups fit per compute unit.
struct ArcPen {
    double arc[4];  // p_f, p_t, q_f, q_t (x's order)
    double cf, ct, ca, dvf, dvt, dva, dq[4];
    int hf, ht;     // positions of the from / to half-edge in the bus-ordered list
};
__device__ __forceinline__ ArcPen arc_pen(const DevModel& m, const ProxRows& rows, const ProxPerm& pm, int l,
                                          const double* s_va, const double* s_hp, const double* s_hq) {
#pragma clang fp contract(off)
    const int L = m.L;
    ArcPen r;
    r.hf = pm.he_pos[l];
    r.ht = pm.he_pos[L + l];
    const int fb = m.f_bus[l], tb = m.t_bus[l];
    const double rate2 = m.rate2[l];
    const double lf = rows.lcon[m.c_thf + l], uf = rows.ucon[m.c_thf + l];
    const double lt = rows.lcon[m.c_tht + l], ut = rows.ucon[m.c_tht + l];
    const double la = rows.lcon[m.c_ang + l], ua = rows.ucon[m.c_ang + l];
    double lo[4], hi[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        lo[a] = rows.lvar[rows.pq0 + a * L + l];
        hi[a] = rows.uvar[rows.pq0 + a * L + l];
    }
    r.arc[0] = s_hp[r.hf];
    r.arc[1] = s_hp[r.ht];
    r.arc[2] = s_hq[r.hf];
    r.arc[3] = s_hq[r.ht];
    r.cf = r.arc[0] * r.arc[0] + r.arc[2] * r.arc[2] - rate2;
    r.ct = r.arc[1] * r.arc[1] + r.arc[3] * r.arc[3] - rate2;
    r.ca = s_va[fb] - s_va[tb];
    r.dvf = viol(r.cf, lf, uf);
    r.dvt = viol(r.ct, lt, ut);
    r.dva = viol(r.ca, la, ua);
#pragma unroll
    for (int a = 0; a < 4; a++) r.dq[a] = viol(r.arc[a], lo[a], hi[a]);
    return r;
}

// LDS (doubles): va, vm [N each]; pg, qg [G each] in the bus-ordered
// generator list's order; p and q of each half-edge [2L each] in the
// bus-ordered half-edge list's order (later the half-edge gradient terms
// d/dva and d/dvm), so that a bus sums one contiguous range; the
// balance-row weights [2N]; the squashing activations [2N + 2G] (z's order)
// and cos, sin of each branch's angle difference [2L], which the gradient
// pass reuses; three partials per wave.  Sums run in the adjacency and
// generator-list orders.
__global__ void __launch_bounds__(kFuseThreads) loss_fused_kernel(DevModel m, ProxBox box, ProxRows rows,
                                                                  ProxPerm pm, const float* __restrict__ z,
                                                                  const double* __restrict__ loads, double rho,
                                                                  double obj_scale, double* __restrict__ loss,
                                                                  double* __restrict__ cvio, double* __restrict__ gz,
                                                                  double* __restrict__ X, double* __restrict__ C,
                                                                  float* __restrict__ dz, double w) {
#pragma clang fp contract(off)
    extern __shared__ double lds[];
    const int N = m.N, L = m.L, G = m.G, D = 2 * N + 2 * G;
    double* s_va = lds;
    double* s_vm = s_va + N;
    double* s_pg = s_vm + N;
    double* s_qg = s_pg + G;
    double* s_hp = s_qg + G;
    double* s_hq = s_hp + 2 * L;
    double* s_wb = s_hq + 2 * L;
    double* s_act = s_wb + 2 * N;
    double* s_cs = s_act + D;
    double* s_red = s_cs + 2 * L;
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const float* zb = z + b * D;
    double* xb = X ? X + b * rows.n : nullptr;
    double* cb = C ? C + b * rows.m : nullptr;
    const double* pdb = loads + b * 2 * N;
    double pen = 0.0, fobj = 0.0, vio = 0.0;

    for (int e = tid; e < D; e += kFuseThreads) {
        const int pos = e < 2 * N ? e : (e < 2 * N + G ? 2 * N + pm.gen_pos[e - 2 * N]
                                                       : 2 * N + G + pm.gen_pos[e - 2 * N - G]);
        double act;
        const double v = squash_entry(box, zb, e, act);
        lds[pos] = v;
        s_act[e < N ? N + e : (e < 2 * N ? e - N : e)] = act;
        if (xb) xb[e] = v;
    }
    __syncthreads();

    // branches: arc flows (and cos, sin for the gradient pass), then the
    // angle and thermal rows and the arc bounds
    for (int l = tid; l < L; l += kFuseThreads) {
        double Cc, Sc;
        const BranchFlows f = branch_flows<true>(m, l, s_va, s_vm, Cc, Sc);
        const int hf = pm.he_pos[l], ht = pm.he_pos[L + l];
        s_cs[l] = Cc;
        s_cs[L + l] = Sc;
        s_hp[hf] = f.pf.F;
        s_hp[ht] = f.pt.F;
        s_hq[hf] = f.qf.F;
        s_hq[ht] = f.qt.F;
        if (xb) {
            xb[rows.pq0 + l] = f.pf.F;
            xb[rows.pq0 + L + l] = f.pt.F;
            xb[rows.pq0 + 2 * L + l] = f.qf.F;
            xb[rows.pq0 + 3 * L + l] = f.qt.F;
        }
    }
    for (int l = tid; l < L; l += kFuseThreads) {  // the same thread's branches: no barrier needed
        const ArcPen r = arc_pen(m, rows, pm, l, s_va, s_hp, s_hq);
        pen += r.dvf * r.dvf;
        pen += r.dvt * r.dvt;
        pen += r.dva * r.dva;
        vio = fmax(vio, fmax(fabs(r.dvf), fmax(fabs(r.dvt), fabs(r.dva))));
#pragma unroll
        for (int a = 0; a < 4; a++) {
            pen += r.dq[a] * r.dq[a];
            vio = fmax(vio, fabs(r.dq[a]));
        }
        if (cb) {  // flow rows: p - F(v) with p := F(v), exactly 0
            cb[m.c_pfr + l] = 0.0;
            cb[m.c_qfr + l] = 0.0;
            cb[m.c_pto + l] = 0.0;
            cb[m.c_qto + l] = 0.0;
            cb[m.c_ang + l] = r.ca;
            cb[m.c_thf + l] = r.cf;
            cb[m.c_tht + l] = r.ct;
        }
    }
    // objective terms and reference rows
    for (int k = tid; k < G; k += kFuseThreads) {
        const double pg = s_pg[pm.gen_pos[k]];
        fobj += m.c2[k] * pg * pg + m.c1[k] * pg + m.c0[k];
    }
    for (int q = tid; q < m.R; q += kFuseThreads) {
        const double c = s_va[m.ref_bus[q]];
        const double dv = viol(c, rows.lcon[m.c_ref + q], rows.ucon[m.c_ref + q]);
        pen += dv * dv;
        vio = fmax(vio, fabs(dv));
        if (cb) cb[m.c_ref + q] = c;
    }
    __syncthreads();

    // buses: balance rows, summed over contiguous half-edge and generator ranges
    for (int i = tid; i < N; i += kFuseThreads) {
        const int h0 = m.adj_ptr[i], h1 = m.adj_ptr[i + 1], g0 = m.gen_ptr[i], g1 = m.gen_ptr[i + 1];
        const double gs = m.gs[i], bs = m.bs[i], pd = pdb[i], qd = pdb[N + i];
        const double lp = rows.lcon[m.c_balp + i], up = rows.ucon[m.c_balp + i];
        const double lq = rows.lcon[m.c_balq + i], uq = rows.ucon[m.c_balq + i];
        const double vm = s_vm[i], v2 = vm * vm;
        double sp = 0.0, sq = 0.0;
        for (int h = h0; h < h1; h++) {
            sp += s_hp[h];
            sq += s_hq[h];
        }
        double cp = pd + gs * v2 + sp, cq = qd - bs * v2 + sq;
        for (int q = g0; q < g1; q++) {
            cp -= s_pg[q];
            cq -= s_qg[q];
        }
        const double dvp = viol(cp, lp, up), dvq = viol(cq, lq, uq);
        pen += dvp * dvp;
        pen += dvq * dvq;
        vio = fmax(vio, fmax(fabs(dvp), fabs(dvq)));
        s_wb[i] = 2.0 * rho * dvp;
        s_wb[N + i] = 2.0 * rho * dvq;
        if (cb) {
            cb[m.c_balp + i] = cp;
            cb[m.c_balq + i] = cq;
        }
    }
    pen = wave_sum64(pen);
    fobj = wave_sum64(fobj);
    vio = wave_max64(vio);
    if ((tid & 63) == 0) {
        s_red[3 * (tid >> 6)] = pen;
        s_red[3 * (tid >> 6) + 1] = fobj;
        s_red[3 * (tid >> 6) + 2] = vio;
    }
    __syncthreads();  // also: every balance weight written, every half-edge value read
    if (tid == 0) {
        double P = 0.0, F = 0.0, V = 0.0;
        for (int w = 0; w < kFuseThreads / 64; w++) {
            P += s_red[3 * w];
            F += s_red[3 * w + 1];
            V = fmax(V, s_red[3 * w + 2]);
        }
        loss[b] = rho * P + obj_scale * F;
        cvio[b] = V;
    }
    if (!gz && !dz) return;

    // branches: d loss / d arc without the balance rows, in place of each
    // branch's own arc values; then with the balance rows, carried through
    // p = F(v) to the branch's four voltage entries, per half-edge
    for (int l = tid; l < L; l += kFuseThreads) {
        const ArcPen r = arc_pen(m, rows, pm, l, s_va, s_hp, s_hq);
        const double wth[2] = {2.0 * rho * r.dvf, 2.0 * rho * r.dvt};
        double ap[4];
#pragma unroll
        for (int a = 0; a < 4; a++) ap[a] = 2.0 * r.arc[a] * wth[a & 1] + 2.0 * rho * r.dq[a];
        s_hp[r.hf] = ap[0];
        s_hp[r.ht] = ap[1];
        s_hq[r.hf] = ap[2];
        s_hq[r.ht] = ap[3];
    }
    for (int l = tid; l < L; l += kFuseThreads) {
        double Cc = s_cs[l], Sc = s_cs[L + l];
        const BranchFlows f = branch_flows<false>(m, l, s_va, s_vm, Cc, Sc);
        const int hf = pm.he_pos[l], ht = pm.he_pos[L + l];
        const double la = rows.lcon[m.c_ang + l], ua = rows.ucon[m.c_ang + l];
        const double wa = 2.0 * rho * viol(s_va[f.fb] - s_va[f.tb], la, ua);
        const double tpf = s_hp[hf] + s_wb[f.fb], tpt = s_hp[ht] + s_wb[f.tb];
        const double tqf = s_hq[hf] + s_wb[N + f.fb], tqt = s_hq[ht] + s_wb[N + f.tb];
        const double gt = tpf * f.pf.Ft + tqf * f.qf.Ft + tpt * f.pt.Ft + tqt * f.qt.Ft;
        s_hp[hf] = gt + wa;
        s_hp[ht] = -(gt + wa);
        s_hq[hf] = tpf * f.pf.Fu + tqf * f.qf.Fu + tpt * f.pt.Fu + tqt * f.qt.Fu;
        s_hq[ht] = tpf * f.pf.Fw + tqf * f.qf.Fw + tpt * f.pt.Fw + tqt * f.qt.Fw;
    }
    __syncthreads();
    // d loss / d z in FP64, or (dz) as (float)(w * d loss / d z): the scaling
    // pass's value written here directly
    auto put = [&](int j, double v) {
        if (dz)
            dz[b * D + j] = (float)(w * v);
        else
            gz[b * D + j] = v;
    };
    for (int i = tid; i < N; i += kFuseThreads) {
        const int h0 = m.adj_ptr[i], h1 = m.adj_ptr[i + 1];
        const double gs = m.gs[i], bs = m.bs[i];
        const double span_v = box.vmax[i] - box.vmin[i];
        const int ref = box.is_ref[i];
        double ga = 0.0, gm = 0.0;
        for (int h = h0; h < h1; h++) {
            ga += s_hp[h];
            gm += s_hq[h];
        }
        const double vm = s_vm[i];
        gm += 2.0 * gs * vm * s_wb[i] - 2.0 * bs * vm * s_wb[N + i];
        const double s = s_act[i];
        put(i, gm * span_v * s * (1.0 - s));
        const double t = s_act[N + i];
        put(N + i, ref ? 0.0 : ga * box.va_span * (1.0 - t * t));
    }
    for (int k = tid; k < G; k += kFuseThreads) {
        const int bus = m.gen_bus[k], q = pm.gen_pos[k];
        const double gp = -s_wb[bus] + obj_scale * (2.0 * m.c2[k] * s_pg[q] + m.c1[k]);
        const double gq = -s_wb[N + bus];
        const double sp = s_act[2 * N + k], sq = s_act[2 * N + G + k];
        put(2 * N + k, gp * (box.pmax[k] - box.pmin[k]) * sp * (1.0 - sp));
        put(2 * N + G + k, gq * (box.qmax[k] - box.qmin[k]) * sq * (1.0 - sq));
    }
}

// dz [B, D] = (float)(w_b * gz[b, j]) with w_b = wb[b], or the constant w
// when wb is NULL
__global__ void scale_rows_kernel(const double* __restrict__ gz, const double* __restrict__ wb, double w, int B,
                                  int D, float* __restrict__ dz) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * D) return;
    dz[idx] = (float)((wb ? wb[idx / D] : w) * gz[idx]);
}

}  // namespace

hipError_t prox_vjp_sum(const double* X, const double* gX1, const double* gX2, const ProxObj& ob, double obj_scale,
                        const double* wb, int B, int64_t n, int64_t nfree, double* gX, hipStream_t s) {
    const int64_t tot = (int64_t)B * n;
    hipLaunchKernelGGL(vjp_sum_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, gX1, gX2, ob, obj_scale,
                       wb, B, n, nfree, gX);
    return hipGetLastError();
}

int prox_gemm_splits(int M, int N, int K) {
    // enough 128 x 128 tiles for one per compute unit, each part at least 4 k tiles
    const int64_t blocks = (int64_t)((M + BM - 1) / BM) * ((N + 127) / 128);
    int s = 1;
    while (blocks * s < 256 && K >= 2 * s * 4 * BK && s < 16) s *= 2;
    return s;
}

namespace {
template <int BN, typename TA, typename TB, typename TACT>
void launch_gemm(int variant, dim3 grid, hipStream_t s, const TA* A, int lda, const TB* B, int ldb, float* C, int ldc,
                 int M, int N, int K, int kchunk, const float* bias, TACT* act, int accumulate, float* part) {
    const dim3 block(GEMM_THREADS);
    switch (variant) {
    case 0: hipLaunchKernelGGL((gemm_kernel<true, true, BN, TA, TB, TACT>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias, act, accumulate, part); break;
    case 1: hipLaunchKernelGGL((gemm_kernel<true, false, BN, TA, TB, TACT>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias, act, accumulate, part); break;
    case 2: hipLaunchKernelGGL((gemm_kernel<false, false, BN, TA, TB, TACT>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias, act, accumulate, part); break;
    default: hipLaunchKernelGGL((gemm_kernel<false, true, BN, TA, TB, TACT>), grid, block, 0, s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias, act, accumulate, part); break;
    }
}

template <typename TA, typename TB, typename TACT>
hipError_t gemm_typed(int variant, const TA* A, int lda, const TB* B, int ldb, float* C, int ldc, int M, int N, int K,
                      const float* bias, TACT* act, int accumulate, int splits, float* work, hipStream_t s,
                      bool finish = true) {
    if (splits < 1) splits = 1;
    const int kchunk = splits == 1 ? K : ((K + splits - 1) / splits + BK - 1) / BK * BK;
    float* part = splits == 1 ? nullptr : work;
    const int my = (M + BM - 1) / BM;
    // 128-column tiles when they already give two workgroups per CU, else
    // 64-column tiles (twice the workgroups, two resident per CU)
    const int64_t wide = (int64_t)my * ((N + 127) / 128) * splits;
    if (wide >= kWideMin)
        launch_gemm<128>(variant, dim3((N + 127) / 128, my, splits), s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias,
                         act, accumulate, part);
    else
        launch_gemm<64>(variant, dim3((N + 63) / 64, my, splits), s, A, lda, B, ldb, C, ldc, M, N, K, kchunk, bias,
                        act, accumulate, part);
    if (splits > 1 && finish) {
        const int64_t tot = (int64_t)M * (N / 4);
        hipLaunchKernelGGL(splitk_sum_kernel<TACT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, work, splits,
                           M, N, C, ldc, bias, act, accumulate);
    }
    return hipGetLastError();
}

template <typename TA, typename TB>
hipError_t gemm_act(int variant, const TA* A, int lda, const TB* B, int ldb, float* C, int ldc, int M, int N, int K,
                    const float* bias, void* act, bool act_bf16, int accumulate, int splits, float* work,
                    hipStream_t s, bool finish = true) {
    if (act_bf16)
        return gemm_typed(variant, A, lda, B, ldb, C, ldc, M, N, K, bias, static_cast<__bf16*>(act), accumulate, splits,
                          work, s, finish);
    return gemm_typed(variant, A, lda, B, ldb, C, ldc, M, N, K, bias, static_cast<float*>(act), accumulate, splits,
                      work, s, finish);
}

template <typename TA>
hipError_t gemm_b(int variant, const TA* A, int lda, const void* B, bool b_bf16, int ldb, float* C, int ldc, int M,
                  int N, int K, const float* bias, void* act, bool act_bf16, int accumulate, int splits, float* work,
                  hipStream_t s, bool finish = true) {
    if (b_bf16)
        return gemm_act(variant, A, lda, static_cast<const __bf16*>(B), ldb, C, ldc, M, N, K, bias, act, act_bf16,
                        accumulate, splits, work, s, finish);
    return gemm_act(variant, A, lda, static_cast<const float*>(B), ldb, C, ldc, M, N, K, bias, act, act_bf16,
                    accumulate, splits, work, s, finish);
}
}  // namespace

namespace {
template <typename TA, typename TB>
hipError_t gelu_bwd_typed(const TA* A, int lda, const TB* B, int ldb, const float* pre, int ldp, __bf16* out, int ldo,
                          int M, int N, int K, float* part, __bf16* outT, int ldT, hipStream_t s) {
    hipLaunchKernelGGL((gemm_gelu_bwd_kernel<true, false, TA, TB>), dim3((N + 63) / 64, (M + BM - 1) / BM, 1),
                       dim3(GEMM_THREADS), 0, s, A, lda, B, ldb, pre, ldp, out, ldo, M, N, K, part, outT, ldT);
    return hipGetLastError();
}
template <typename TA>
hipError_t gelu_bwd_b(const TA* A, int lda, const void* B, bool b_bf16, int ldb, const float* pre, int ldp, __bf16* out,
                      int ldo, int M, int N, int K, float* part, __bf16* outT, int ldT, hipStream_t s) {
    if (b_bf16)
        return gelu_bwd_typed(A, lda, static_cast<const __bf16*>(B), ldb, pre, ldp, out, ldo, M, N, K, part, outT,
                              ldT, s);
    return gelu_bwd_typed(A, lda, static_cast<const float*>(B), ldb, pre, ldp, out, ldo, M, N, K, part, outT, ldT,
                          s);
}
}  // namespace

hipError_t prox_gemm_gelu_bwd(const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                              const float* pre, int ldp, void* out, int ldo, int M, int N, int K, float* part,
                              hipStream_t s, void* outT, int ldT) {
    __bf16* o = static_cast<__bf16*>(out);
    __bf16* oT = static_cast<__bf16*>(outT);
    if (a_bf16)
        return gelu_bwd_b(static_cast<const __bf16*>(A), lda, B, b_bf16, ldb, pre, ldp, o, ldo, M, N, K, part, oT, ldT,
                          s);
    return gelu_bwd_b(static_cast<const float*>(A), lda, B, b_bf16, ldb, pre, ldp, o, ldo, M, N, K, part, oT, ldT, s);
}

hipError_t prox_colsum_parts(const float* part, int chunks, int N, float* out, float scale, hipStream_t s) {
    hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 63) / 64), dim3(256), 0, s, part, chunks, N, out, scale);
    return hipGetLastError();
}

hipError_t prox_gemm_mixed(int variant, const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                           float* C, int ldc, int M, int N, int K, const float* bias, void* act, bool act_bf16,
                           int accumulate, int splits, float* work, hipStream_t s) {
    if (a_bf16)
        return gemm_b(variant, static_cast<const __bf16*>(A), lda, B, b_bf16, ldb, C, ldc, M, N, K, bias, act, act_bf16,
                      accumulate, splits, work, s);
    return gemm_b(variant, static_cast<const float*>(A), lda, B, b_bf16, ldb, C, ldc, M, N, K, bias, act, act_bf16,
                  accumulate, splits, work, s);
}

hipError_t prox_gemm_split_parts(int variant, const void* A, bool a_bf16, int lda, const void* B, bool b_bf16, int ldb,
                                 int M, int N, int K, int splits, float* work, hipStream_t s) {
    if (a_bf16)
        return gemm_b(variant, static_cast<const __bf16*>(A), lda, B, b_bf16, ldb, nullptr, N, M, N, K, nullptr, nullptr,
                      false, 0, splits, work, s, false);
    return gemm_b(variant, static_cast<const float*>(A), lda, B, b_bf16, ldb, nullptr, N, M, N, K, nullptr, nullptr,
                  false, 0, splits, work, s, false);
}

hipError_t prox_wgrad_finish(const float* work, int splits, int M, int N, float* C, int ldc, const float* part,
                             int chunks, int NB, float* bias_out, hipStream_t s) {
    const int nsum = (int)(((int64_t)M * (N / 4) + 255) / 256);
    hipLaunchKernelGGL(wgrad_finish_kernel, dim3((unsigned)(nsum + (NB + 63) / 64)), dim3(256), 0, s, work, splits, M,
                       N, C, ldc, nsum, part, chunks, NB, bias_out);
    return hipGetLastError();
}

hipError_t prox_gemm(int variant, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int M, int N,
                     int K, const float* bias, float* act, int accumulate, int splits, float* work, hipStream_t s) {
    return prox_gemm_mixed(variant, A, false, lda, B, false, ldb, C, ldc, M, N, K, bias, act, false, accumulate, splits,
                           work, s);
}

hipError_t prox_gelu_bwd(const float* pre, const float* dact, float* dpre, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gelu_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pre, dact, dpre, n);
    return hipGetLastError();
}

hipError_t prox_colsum_first(const float* X, int M, int N, float* part, hipStream_t s) {
    const int chunks = (M + COLSUM_ROWS - 1) / COLSUM_ROWS;
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0, s, X, M, N, part);
    return hipGetLastError();
}

hipError_t prox_colsum(const float* X, int M, int N, float* part, float* out, float scale, hipStream_t s) {
    const int chunks = (M + COLSUM_ROWS - 1) / COLSUM_ROWS;
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0, s, X, M, N, part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 63) / 64), dim3(256), 0, s, part, chunks, N, out, scale);
    return hipGetLastError();
}


hipError_t prox_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                     int step, void* pb, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m1, m2, n, lr, b1, b2,
                       eps, c1, c2, static_cast<__bf16*>(pb));
    return hipGetLastError();
}

hipError_t prox_adam_dev(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                         float eps, int32_t* step, void* pb, hipStream_t s) {
    auto a16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (a16(p) && a16(g) && a16(m1) && a16(m2) && (reinterpret_cast<uintptr_t>(pb) & 7u) == 0) {
        const int64_t blocks = std::min<int64_t>((n / 4 + 255) / 256, 2048);
        hipLaunchKernelGGL(adam_dev4_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, p, g, m1,
                           m2, n, lr, b1, b2, eps, step, static_cast<__bf16*>(pb));
    } else {
        hipLaunchKernelGGL(adam_dev_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m1, m2, n, lr,
                           b1, b2, eps, step, static_cast<__bf16*>(pb));
    }
    hipLaunchKernelGGL(step_bump_kernel, dim3(1), dim3(1), 0, s, step);
    return hipGetLastError();
}

hipError_t prox_to_bf16(const float* x, int64_t n, void* y, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, static_cast<__bf16*>(y));
    return hipGetLastError();
}

hipError_t prox_squash_fwd(const float* z, int B, const ProxBox& box, double* X, int64_t n, bool arcs, hipStream_t s) {
    const int64_t per = arcs ? n : 2 * (int64_t)box.N + 2 * box.G;
    const int64_t tot = (int64_t)B * per;
    hipLaunchKernelGGL(squash_fwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, B, box, X, n, per);
    return hipGetLastError();
}

hipError_t prox_squash_bwd(const float* z, int B, const ProxBox& box, const double* gX1, const double* gX2,
                           const double* gObj, double obj_scale, int64_t n, float* dz, float scale, hipStream_t s) {
    const int64_t tot = (int64_t)B * (2 * box.N + 2 * box.G);
    hipLaunchKernelGGL(squash_bwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, B, box, gX1, gX2,
                       gObj, obj_scale, n, dz, scale);
    return hipGetLastError();
}

hipError_t prox_loss_bwd(const float* z, int B, const ProxBox& box, const ProxObj& ob, const double* X,
                         const double* gX1, double obj_scale, const double* wb, int64_t n, float* dz, hipStream_t s) {
    const int64_t tot = (int64_t)B * (2 * box.N + 2 * box.G);
    hipLaunchKernelGGL(loss_bwd_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, B, box, ob, X, gX1,
                       obj_scale, wb, n, dz);
    return hipGetLastError();
}

hipError_t prox_penalty(const double* C, const double* X, const double* F, double obj_scale, const ProxRows& rows,
                        double rho, int B, double* pen, double* cvio, double* W, double* gpq, int vjp, hipStream_t s) {
    const size_t lds = gpq ? 0 : sizeof(double) * (size_t)rows.npq;
    hipLaunchKernelGGL(penalty_kernel, dim3(B), dim3(256), lds, s, C, X, F, obj_scale, rows, rho, pen, cvio, W, gpq,
                       vjp);
    return hipGetLastError();
}

hipError_t prox_vjp_weights(const double* X, const double* W, const double* gpq, const ProxRows& rows, int B,
                            double* Wt, hipStream_t s) {
    if (Wt != W) {
        const int64_t tot = (int64_t)B * rows.m;
        hipLaunchKernelGGL(copy_off_flow_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, rows, B, Wt);
    }
    const int64_t nfl = (int64_t)B * (rows.flow1 - rows.flow0);
    if (nfl > 0)
        hipLaunchKernelGGL(vjp_weights_kernel, dim3((unsigned)((nfl + 255) / 256)), dim3(256), 0, s, X, W, gpq, rows,
                           B, Wt);
    return hipGetLastError();
}


size_t prox_loss_fused_lds(int N, int L, int G) {
    return sizeof(double) * ((size_t)6 * N + 4 * (size_t)G + 6 * (size_t)L + 3 * (kFuseThreads / 64));
}

hipError_t prox_loss_fused(const DevModel& m, const ProxBox& box, const ProxRows& rows, const ProxPerm& pm,
                           const float* z, const double* loads, int B, double rho, double obj_scale, double* loss,
                           double* cvio, double* gz, double* X, double* C, hipStream_t s, float* dz, double w) {
    hipLaunchKernelGGL(loss_fused_kernel, dim3(B), dim3(kFuseThreads), prox_loss_fused_lds(m.N, m.L, m.G), s, m, box,
                       rows, pm, z, loads, rho, obj_scale, loss, cvio, gz, X, C, dz, w);
    return hipGetLastError();
}

hipError_t prox_sample_loads(const double* r, const double* base, const double* inv_scale, double spread, int B,
                             int N, double* loads, float* feats, hipStream_t s) {
    const int64_t tot = (int64_t)B * 2 * N;
    hipLaunchKernelGGL(sample_loads_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, r, base, inv_scale,
                       spread, B, N, loads, feats);
    return hipGetLastError();
}

hipError_t prox_scale_rows(const double* gz, const double* wb, double w, int B, int D, float* dz, hipStream_t s) {
    const int64_t tot = (int64_t)B * D;
    hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, gz, wb, w, B, D, dz);
    return hipGetLastError();
}

}  // namespace opf
