// Block-level complex GEMM core used by the Theta, Gram, split and measurement
// kernels.  One 256-thread workgroup computes a BM x BN tile of
//     C(m, n) = sum_k A(m, k) * B(k, n)
// where A and B are supplied by load functors (so transposition, conjugation,
// row weights and gathered physical indices cost nothing extra) and the result
// is handed to a store functor.  Operand tiles are staged through LDS; each
// thread owns a 4 x 4 block of outputs spread with stride 16 (conflict-free LDS
// reads).  A_KFAST / B_NFAST select the global-load order so that consecutive
// lanes touch consecutive addresses for the operand's storage order.
#pragma once
#include "common.h"

template <class Acc, bool A_KFAST, bool B_NFAST, int BK, class LA, class LB, class SC>
__device__ __forceinline__ void block_gemm(int M, int N, int K, int m0, int n0, LA la, LB lb, SC sc,
                                           Acc* As /* BK*64 */, Acc* Bs /* BK*64 */)
{
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    Acc acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = czero<Acc>();

    for (int k0 = 0; k0 < K; k0 += BK) {
        // A tile -> As[kk*64 + mm]
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
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            Acc a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk * 64 + ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk * 64 + tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) cfma(acc[r][c], a[r], b[c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int gm = m0 + ty + 16 * r, gn = n0 + tx + 16 * c;
            if (gm < M && gn < N) sc(gm, gn, acc[r][c]);
        }
}
