// Block-level complex GEMM core used by the Theta, Gram, split and measurement
// kernels.  Complex64 operands run on the FP32 matrix cores (block_gemm_mfma_c32, FP32 sums per
// k-chunk added in FP64), complex128 operands on the FP64 matrix cores (block_gemm_mfma_c64).
// Both hand FP64 sums (double2) to the store functor.  One 256-thread workgroup computes a
// 64 x 64 tile of
//     C(m, n) = sum_k A(m, k) * B(k, n)
// where A and B are supplied by load functors (so transposition, conjugation,
// row weights and gathered physical indices cost nothing extra) and the result
// is handed to a store functor.  Operand tiles are staged through LDS.  A_KFAST / B_NFAST
// select the global-load order so that consecutive lanes touch consecutive addresses for the
// operand's storage order.
#pragma once
#include <type_traits>
#include "common.h"

typedef float gemm_f4 __attribute__((ext_vector_type(4)));

template <class Acc, bool A_KFAST, bool B_NFAST, int BK, class LA, class LB>
__device__ __forceinline__ void gemm_stage(int M, int N, int K, int m0, int n0, int k0, LA la, LB lb, Acc* As,
                                           Acc* Bs) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int e0 = 0; e0 < 64 * BK; e0 += 256) {
        int e = e0 + tid;
        int mm, kk;
        if (A_KFAST) { mm = e / BK; kk = e % BK; } else { kk = e / 64; mm = e % 64; }
        int gm = m0 + mm, gk = k0 + kk;
        As[kk * 64 + mm] = (gm < M && gk < K) ? la(gm, gk) : czero<Acc>();
    }
#pragma unroll
    for (int e0 = 0; e0 < 64 * BK; e0 += 256) {
        int e = e0 + tid;
        int nn, kk;
        if (B_NFAST) { kk = e / 64; nn = e % 64; } else { nn = e / BK; kk = e % BK; }
        int gn = n0 + nn, gk = k0 + kk;
        Bs[kk * 64 + nn] = (gn < N && gk < K) ? lb(gk, gn) : czero<Acc>();
    }
}

typedef double gemm_d4 __attribute__((ext_vector_type(4)));

// Complex64 tiles on the matrix cores: each of the 4 waves owns a 32 x 32 quarter of the
// 64 x 64 tile as 2 x 2 blocks of 16 x 16; a k-step of 4 is four real MFMA 16x16x4 f32
// products per block (re*re, -im*im into the real part, re*im, im*re into the imaginary part).
// The products of one staged k-chunk (BK deep) accumulate in FP32 on the matrix cores, and each
// chunk's sums are added to FP64 accumulators: a K-deep sum then rounds like BK-deep FP32 sums
// added exactly, about sqrt(K / BK) times less than one K-deep FP32 accumulation.  The store
// functor receives the FP64 sums.  Operand layouts: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is C[4*(l/16) + r][l%16].
// The store runs in PASSES passes over row halves (PASSES 2: waves 0-1 hold tile rows 0-31, waves
// 2-3 rows 32-63); ep(pass) is called by every thread after each pass, so a kernel can stage half
// the output tile in LDS at a time.
struct NoEpilogue {
    __device__ void operator()(int) const {}
};

template <bool A_KFAST, bool B_NFAST, int BK, int PASSES = 1, class LA, class LB, class SC, class EP = NoEpilogue>
__device__ __forceinline__ void block_gemm_mfma_c32(int M, int N, int K, int m0, int n0, LA la, LB lb, SC sc,
                                                    float2* As, float2* Bs, EP ep = EP{}) {
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    gemm_d4 dr[2][2], di[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            dr[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
            di[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
        }
    for (int k0 = 0; k0 < K; k0 += BK) {
        gemm_stage<float2, A_KFAST, B_NFAST, BK>(M, N, K, m0, n0, k0, la, lb, As, Bs);
        __syncthreads();
        gemm_f4 cr[2][2], ci[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = gemm_f4{0.f, 0.f, 0.f, 0.f};
                ci[a][b] = gemm_f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float2 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[(kk + lk) * 64 + wm + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[(kk + lk) * 64 + wn + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                    cr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[a].y, bv[b].y, cr[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    dr[a][b][r] += (double)cr[a][b][r];
                    di[a][b][r] += (double)ci[a][b][r];
                }
    }
    for (int pass = 0; pass < PASSES; ++pass) {
        if (PASSES == 1 || (wv >> 1) == pass) {  // uniform per wave
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gm = m0 + wm + 16 * a + 4 * lk + r, gn = n0 + wn + 16 * b + li;
                        if (gm < M && gn < N) sc(gm, gn, make_double2(dr[a][b][r], di[a][b][r]));
                    }
        }
        ep(pass);
    }
}


// Complex128 tiles on the FP64 matrix cores, the same wave and block split as the FP32 core: a
// k-step of 4 is four real MFMA 16x16x4 f64 products per 16 x 16 block, accumulated in FP64.
// Operand layouts as above (lane l supplies A[l%16][l/16] and B[l/16][l%16]); accumulator element
// r of lane l is C[l/16 + 4*r][l%16].
template <bool A_KFAST, bool B_NFAST, int BK, int PASSES = 1, class LA, class LB, class SC, class EP = NoEpilogue>
__device__ __forceinline__ void block_gemm_mfma_c64(int M, int N, int K, int m0, int n0, LA la, LB lb, SC sc,
                                                    double2* As, double2* Bs, EP ep = EP{}) {
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    gemm_d4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
            ci[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
        }
    for (int k0 = 0; k0 < K; k0 += BK) {
        gemm_stage<double2, A_KFAST, B_NFAST, BK>(M, N, K, m0, n0, k0, la, lb, As, Bs);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double2 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[(kk + lk) * 64 + wm + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[(kk + lk) * 64 + wn + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[b].y, cr[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    for (int pass = 0; pass < PASSES; ++pass) {
        if (PASSES == 1 || (wv >> 1) == pass) {  // uniform per wave
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gm = m0 + wm + 16 * a + lk + 4 * r, gn = n0 + wn + 16 * b + li;
                        if (gm < M && gn < N) sc(gm, gn, make_double2(cr[a][b][r], ci[a][b][r]));
                    }
        }
        ep(pass);
    }
}

template <class Acc, bool A_KFAST, bool B_NFAST, int BK, int PASSES = 1, class LA, class LB, class SC,
          class EP = NoEpilogue>
__device__ __forceinline__ void block_gemm(int M, int N, int K, int m0, int n0, LA la, LB lb, SC sc,
                                           Acc* As /* BK*64 */, Acc* Bs /* BK*64 */, EP ep = EP{}) {
    static_assert(BK % 4 == 0, "MFMA k-steps of 4");
    if constexpr (std::is_same<Acc, float2>::value)
        block_gemm_mfma_c32<A_KFAST, B_NFAST, BK, PASSES>(M, N, K, m0, n0, la, lb, sc, As, Bs, ep);
    else
        block_gemm_mfma_c64<A_KFAST, B_NFAST, BK, PASSES>(M, N, K, m0, n0, la, lb, sc, As, Bs, ep);
}
