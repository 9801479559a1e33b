// Two-site TEBD update kernels (gfx950).
//
// One Trotter layer is a set of independent work items (instance b, bond) --
// all bonds of one parity of every unmasked instance commute (Sec. 2.3).  Each
// item goes through
//   k_theta_gate  Theta~ = G (x) (B_bond . B_{bond+1})  (complex GEMM with the gate applied to the
//             staged output tile, eq. Theta / eq. ThetaPurified; plain k_theta for centre shifts)
//   k_gram    H = Theta~^+ diag(Lambda_{bond-1}^2) Theta~   (FP64, lower triangle; k_gram_mfma on
//             the FP64 matrix cores for 64 < n <= 128)
//   k_hetrd   Householder reduction H = Q T Q^+, T real tridiagonal (FP64; k_hetrd_mfma head and
//             tail launches for n <= 128)
//   k_steqr   implicit QL on T, logging every Givens rotation (FP64)
//   k_select  sort eigenvalues, truncation rank, discarded weight (eq. HilbertSchmidtNorm)
//   k_vecs    replay the rotations on the selected unit vectors, back-transform by Q,
//             store B_{bond+1} <- V^+ (right isometry)
//   k_split   B_bond <- Theta~ V / s  (Hastings split), dims, log s and weight per item
// In split mode with n <= 128 and chi <= 64, k_bisect (eigenvalues by Sturm counts) and k_tvecs
// (twisted-factorization eigenvectors, blocked back-transformation on the matrix cores) replace
// k_steqr, k_select and k_vecs; k_steqr_fb, k_select and k_vecs_fast then run only for items
// holding a degenerate multiplet.  In FP64 mode every eigenvector is formed and a one-sided
// Jacobi refinement (k_jac_y, k_jacobi, k_select mode 2, k_jac_store) replaces the last two steps.
// The eigenvalues of H are the squared singular values of Theta = Lambda Theta~ and
// its eigenvectors the right singular vectors, so this is the truncated SVD of the
// two-site update computed in FP64 without ever forming U.
#include "common.h"
#include "gemm.h"
#include <float.h>

#define NT 256
// four doubles: one lane's share of a 16 x 16 FP64 MFMA accumulator (rows l/16 + 4 e, column l%16)
typedef double hm_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int tri(int r, int c) { return (r * (r + 1)) / 2 + c; }

// value of v in lane `lane` (uniform index) broadcast to the wave without an LDS round trip
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wavefront (every lane receives the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct ItemDims { int b, bond, chil, chim, chir, dl, dr, m, n; };

__device__ __forceinline__ bool item_dims(const DevState& s, const DevWork& w, int j, ItemDims& d) {
    if (j >= w.nitems) return false;
    if (!item_coords(w, j, d.b, d.bond)) return false;
    d.chil = bond_dim(s, d.b, d.bond);
    d.chim = bond_dim(s, d.b, d.bond + 1);
    d.chir = bond_dim(s, d.b, d.bond + 2);
    d.dl = s.dsite[d.bond];
    d.dr = s.dsite[d.bond + 1];
    d.m = d.chil * d.dl;
    d.n = d.dr * d.chir;
    return true;
}

// ------------------------------------------------------------------ Theta
// T: storage type of the site tensors.  TC: operand type of the contraction, complex64 on the FP32
// matrix cores (FP32 sums per 8-deep k-chunk, added in FP64) or complex128 on the FP64 ones (the
// products of complex64 values are exact there).  Theta~ goes to the workspace in complex128 in
// both cases, so it is not rounded again before the Gram matrix and the split read it.
template <class T, class TC>
__global__ __launch_bounds__(NT) void k_theta(DevState s, DevWork w, int tiles_n) {
    __shared__ TC As[8 * 64], Bs[8 * 64];
    ItemDims d;
    if (!item_dims(s, w, blockIdx.y, d)) return;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= d.m || tn * 64 >= d.n) return;
    const T* P = site_ptr<T>(s, d.b, d.bond);
    const T* Q = site_ptr<T>(s, d.b, d.bond + 1);
    double2* out = reinterpret_cast<double2*>(w.theta) + (size_t)blockIdx.y * w.theta_stride;
    const int K = d.chim, n = d.n;
    block_gemm<TC, true, true, 8>(
        d.m, d.n, K, tm * 64, tn * 64,
        [&](int r, int k) { return cconv<TC>(P[(size_t)r * K + k]); },
        [&](int k, int c) { return cconv<TC>(Q[(size_t)k * n + c]); },
        [&](int r, int c, double2 v) { out[(size_t)r * n + c] = v; }, As, Bs);
}

// Theta~ = G (x) (B_bond . B_{bond+1}) in one pass (eq. Theta): the GEMM runs over a virtual
// column numbering in which a 64-wide tile holds cw = 64/d_r values of c for every q (column
// V -> q = (V % 64) / cw, c = (V / 64) cw + (V % 64) % cw), so the d_l d_r entries that the gate
// mixes, rows (a, p) and columns (q, c), all land in one tile.  The tile is staged in LDS and
// the gate applied on the way to memory.
template <class T, class TC, int DM>
__global__ __launch_bounds__(NT, DM <= 4 ? 4 : 2) void k_theta_gate(DevState s, DevWork w, int tiles_n) {
    // Half of the output tile (32 rows, FP64) is staged at a time and reuses the operand staging
    // space: block_gemm ends its k loop with a barrier, after which the staging buffers are dead.
    // With 36 KB of LDS and, for d_l d_r <= 4, the launch bound (at most 128 registers, no spills)
    // four workgroups share a CU (the whole tile in LDS allowed two).
    __shared__ double2 smem[32 * 64];
    __shared__ double2 G[256];
    TC* As = reinterpret_cast<TC*>(smem);
    TC* Bs = As + 8 * 64;
    double2* tile = smem;
    ItemDims d;
    if (!item_dims(s, w, blockIdx.y, d)) return;
    const int dl = d.dl, dr = d.dr, D = dl * dr, cw = 64 / dr, chir = d.chir, n = d.n;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= d.m || tn * cw >= chir) return;
    // the gate is staged as G - 1 and the identity part added exactly, in FP64: a Trotter gate is
    // 1 + O(dt), and rounding G itself to FP32 would perturb the generator by ~eps/dt coherently
    // at every step
    const double2* g = w.gates + (size_t)d.bond * w.gstride;
    for (int e = threadIdx.x; e < D * D; e += NT) {
        double2 ge = g[e];
        if (e / D == e % D) ge.x -= 1.0;
        G[e] = ge;
    }
    const T* P = site_ptr<T>(s, d.b, d.bond);
    const T* Q = site_ptr<T>(s, d.b, d.bond + 1);
    double2* out = reinterpret_cast<double2*>(w.theta) + (size_t)blockIdx.y * w.theta_stride;
    const int K = d.chim, m0 = tm * 64;
    // rows (a, p) of one pair never straddle the halves: 32 is a multiple of d_l (<= 8)
    const auto gate_half = [&](int pass) {
        __syncthreads();  // the half's entries are in LDS
        const int h0 = m0 + 32 * pass;
        const int npair = (32 / dl) * cw;
        for (int e = threadIdx.x; e < npair; e += NT) {
            const int al = e / cw, cl = e % cw, c = tn * cw + cl;
            const int r0 = h0 + al * dl;
            if (c >= chir || r0 >= d.m) continue;
            double2 v[DM];
#pragma unroll
            for (int x = 0; x < DM; ++x)
                if (x < D) v[x] = tile[(al * dl + x / dr) * 64 + (x % dr) * cw + cl];
#pragma unroll
            for (int o = 0; o < DM; ++o) {
                if (o < D) {
                    double2 acc = v[o];
#pragma unroll
                    for (int x = 0; x < DM; ++x)
                        if (x < D) cfma(acc, G[o * D + x], v[x]);
                    out[(size_t)(r0 + o / dr) * n + (o % dr) * chir + c] = acc;
                }
            }
        }
        __syncthreads();  // the half is consumed before the next one is stored
    };
    block_gemm<TC, true, true, 8, 2>(
        d.m, tiles_n * 64, K, m0, tn * 64,
        [&](int r, int k) { return cconv<TC>(P[(size_t)r * K + k]); },
        [&](int k, int V) {
            const int loc = V & 63, q = loc / cw, c = (V >> 6) * cw + loc % cw;
            return c < chir ? cconv<TC>(Q[(size_t)k * n + q * chir + c]) : czero<TC>();
        },
        [&](int r, int V, double2 v) { tile[((r - m0) & 31) * 64 + (V & 63)] = v; }, As, Bs, gate_half);
}

// ------------------------------------------------------------------ weighted Gram (FP64)
template <class T>
__global__ __launch_bounds__(NT) void k_gram(DevState s, DevWork w, int tiles_n) {
    __shared__ double2 As[8 * 64], Bs[8 * 64];
    ItemDims d;
    if (!item_dims(s, w, blockIdx.y, d)) return;
    if (w.qr_route && d.m < d.n) return;  // built by k_qr_wide instead
    if (blockIdx.x == 0 && threadIdx.x == 0) w.gsz[blockIdx.y] = d.n;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= d.n || tn * 64 >= d.n || tm < tn) return;  // lower block triangle only
    const T* th = reinterpret_cast<const T*>(w.theta) + (size_t)blockIdx.y * w.theta_stride;
    const double* lamL = (d.bond > 0 && !w.unitw) ? lam_ptr(s, d.b, d.bond - 1) : nullptr;
    const int n = d.n, dl = d.dl;
    double2* G = w.gram + (size_t)blockIdx.y * w.nmax * w.nmax;
    block_gemm<double2, false, true, 8>(
        n, n, d.m, tm * 64, tn * 64,
        [&](int i, int r) { return cconj(cconv<double2>(th[(size_t)r * n + i])); },
        [&](int r, int c) {
            double wl = 1.0;
            if (lamL) { double l = lamL[r / dl]; wl = l * l; }
            return cscale(cconv<double2>(th[(size_t)r * n + c]), wl);
        },
        [&](int i, int c, double2 v) { G[(size_t)i * n + c] = v; }, As, Bs);
}


// ------------------------------------------------------------------ QR route for wide Theta (FP64 mode)
// For m < n the n x n Gram matrix has rank <= m and its top-m eigenvectors would have to be
// separated from rounding noise.  Instead: Householder QR  Theta^+ = Q R  (Q = H_0 ... H_{m-1},
// R m x m), the m x m Hermitian problem  R R^+ = W diag W^+  (the usual eigen pipeline), and
// V = Q [W; 0], whose columns span the row space of Theta exactly.
// Weighted Gram H = Theta~^+ diag(w) Theta~ for n <= 128 on the FP64 matrix cores, one item per
// 256-thread workgroup, w_r = Lambda_{b-1}[r / d_l]^2.  The 36 lower 16 x 16 tiles of H stay in MFMA
// accumulators: wave q owns the tile rows q and 7 - q (q + 1 and 8 - q tiles, nine per wave).
// Slot s of a wave is the tile (q, s) for s <= q, else (7 - q, s - q - 1).  Theta~ streams through
// LDS in chunks of 16 rows, double-buffered (the next chunk's entries load into registers during
// the current chunk's products, so a chunk costs one barrier).  Per 4-row step, lane l supplies
// the A operand w_r Theta~[r][16 ti + l%16] of its tile row and the B operand Theta~[r][16 tj + l%16]
// of each tile, r = 4-row base + l/16; conj(A) B is four real 16x16x4 products.
#define GM_RC 16
template <class T>
__global__ __launch_bounds__(NT, 2) void k_gram_mfma(DevState s, DevWork w) {
    static_assert(NT == 256, "four waves, two tile rows each");
    __shared__ T ts[2][GM_RC * 128];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (w.qr_route && d.m < d.n) return;  // built by k_qr_wide instead
    const int tid = threadIdx.x;
    if (tid == 0) w.gsz[j] = d.n;
    const int n = d.n, m = d.m, dl = d.dl;
    const T* th = reinterpret_cast<const T*>(w.theta) + (size_t)j * w.theta_stride;
    const double* lamL = (d.bond > 0 && !w.unitw) ? lam_ptr(s, d.b, d.bond - 1) : nullptr;
    const int wv = tid >> 6, lane = tid & 63, g = lane >> 4, cl = lane & 15;
    const int ra = wv, rb = 7 - wv;  // this wave's tile rows
    hm_d4 gre[9], gim[9];
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
        gre[sl] = hm_d4{0.0, 0.0, 0.0, 0.0};
        gim[sl] = hm_d4{0.0, 0.0, 0.0, 0.0};
    }
    const int nch = (m + GM_RC - 1) / GM_RC;
    constexpr int PER = GM_RC * 128 / NT;  // chunk entries per thread: row e / 128, column e % 128
    T pf[PER];
    const auto load_chunk = [&](int ch) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + NT * u, r = ch * GM_RC + e / 128, c = e % 128;
            pf[u] = (r < m && c < n) ? th[(size_t)r * n + c] : T{};
        }
    };
    if (nch > 0) load_chunk(0);
    for (int ch = 0; ch < nch; ++ch) {
        T* buf = ts[ch & 1];
#pragma unroll
        for (int u = 0; u < PER; ++u) buf[tid + NT * u] = pf[u];
        __syncthreads();  // also: every wave is done with the chunk that used this buffer before
        if (ch + 1 < nch) load_chunk(ch + 1);
#pragma unroll
        for (int q4 = 0; q4 < GM_RC / 4; ++q4) {
            const int rl = 4 * q4 + g, r = ch * GM_RC + rl;
            double wl = 1.0;
            if (lamL && r < m) {
                const double l = lamL[r / dl];
                wl = l * l;
            }
            double2 xa = cconv<double2>(buf[rl * 128 + 16 * ra + cl]);
            double2 xb = cconv<double2>(buf[rl * 128 + 16 * rb + cl]);
            xa = mk(wl * xa.x, wl * xa.y);
            xb = mk(wl * xb.x, wl * xb.y);
#pragma unroll
            for (int sl = 0; sl < 9; ++sl) {
                const bool inA = sl <= ra;  // uniform per wave
                const int ti = inA ? ra : rb, tj = inA ? sl : sl - ra - 1;
                if (16 * ti < n) {  // uniform
                    double ax = xa.x, ay = xa.y;
                    ax = inA ? ax : xb.x;
                    ay = inA ? ay : xb.y;
                    const double2 bv = cconv<double2>(buf[rl * 128 + 16 * tj + cl]);
                    // conj(a) b: re = ax bx + ay by, im = ax by - ay bx
                    gre[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bv.x, gre[sl], 0, 0, 0);
                    gre[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, bv.y, gre[sl], 0, 0, 0);
                    gim[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bv.y, gim[sl], 0, 0, 0);
                    gim[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, bv.x, gim[sl], 0, 0, 0);
                }
            }
        }
    }
    double2* G = w.gram + (size_t)j * w.nmax * w.nmax;
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
        const bool inA = sl <= ra;
        const int ti = inA ? ra : rb, tj = inA ? sl : sl - ra - 1;
        const int c = 16 * tj + cl;
        if (16 * ti < n && c < n) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * ti + g + 4 * e;
                if (i < n) G[(size_t)i * n + c] = mk(gre[sl][e], gim[sl][e]);
            }
        }
    }
}

__global__ __launch_bounds__(NT) void k_qr_wide(DevState s, DevWork w) {
    __shared__ double red[NT / 64];
    __shared__ double2 sh_tau, sh_sc;
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (!(d.m < d.n)) return;
    const int m = d.m, n = d.n, tid = threadIdx.x;
    const double2* th = reinterpret_cast<const double2*>(w.theta) + (size_t)j * w.theta_stride;
    const double* lamL = (d.bond > 0 && !w.unitw) ? lam_ptr(s, d.b, d.bond - 1) : nullptr;
    double2* A = w.qra + (size_t)j * w.nmax * w.nmax;   // n x m, row-major, ld = m
    double2* qt = w.qtau + (size_t)j * w.nmax;
    // A[r][c] = conj(Theta[c][r]), Theta = Lambda_left Theta~
    for (int e = tid; e < n * m; e += NT) {
        int r = e / m, c = e % m;
        double wl = lamL ? lamL[c / d.dl] : 1.0;
        A[e] = cscale(cconj(th[(size_t)c * n + r]), wl);
    }
    __syncthreads();
    for (int jj = 0; jj < m; ++jj) {
        double p = 0.0;
        for (int r = jj + 1 + tid; r < n; r += NT) {
            double2 x = A[(size_t)r * m + jj];
            p += x.x * x.x + x.y * x.y;
        }
        p = wave_sum(p);
        if ((tid & 63) == 0) red[tid >> 6] = p;
        __syncthreads();
        if (tid == 0) {
            double xn2 = red[0] + red[1] + red[2] + red[3];
            double2 alpha = A[(size_t)jj * m + jj];
            double2 t, sc;
            double beta;
            if (xn2 == 0.0 && alpha.y == 0.0) {
                t = mk(0.0, 0.0);
                beta = alpha.x;
                sc = mk(1.0, 0.0);
            } else {
                double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                t = mk((beta - alpha.x) / beta, -alpha.y / beta);
                double2 z = mk(alpha.x - beta, alpha.y);
                double den = z.x * z.x + z.y * z.y;
                sc = mk(z.x / den, -z.y / den);
            }
            sh_tau = t;
            sh_sc = sc;
            qt[jj] = t;
            A[(size_t)jj * m + jj] = mk(beta, 0.0);  // R[jj][jj]; v[0] = 1 is implicit
        }
        __syncthreads();
        const double2 t = sh_tau, sc = sh_sc;
        for (int r = jj + 1 + tid; r < n; r += NT) A[(size_t)r * m + jj] = cmul(A[(size_t)r * m + jj], sc);
        __syncthreads();
        if (t.x != 0.0 || t.y != 0.0) {
            // A[jj:, c] <- (I - conj(tau) v v^+) A[jj:, c] for c > jj; one thread per column
            const double2 tc = cconj(t);
            for (int c = jj + 1 + tid; c < m; c += NT) {
                double2 acc = A[(size_t)jj * m + c];  // v[0] = 1
                for (int r = jj + 1; r < n; ++r) cfmac(acc, A[(size_t)r * m + jj], A[(size_t)r * m + c]);
                acc = cmul(tc, acc);
                double2 a0 = A[(size_t)jj * m + c];
                A[(size_t)jj * m + c] = csub(a0, acc);
                for (int r = jj + 1; r < n; ++r) {
                    double2 u = cmul(A[(size_t)r * m + jj], acc);
                    A[(size_t)r * m + c] = csub(A[(size_t)r * m + c], u);
                }
            }
        }
        __syncthreads();
    }
    // Hermitian problem R R^+ (m x m) into the Gram slot (full matrix)
    double2* G = w.gram + (size_t)j * w.nmax * w.nmax;
    for (int e = tid; e < m * m; e += NT) {
        int a = e / m, b2 = e % m;
        double2 acc = mk(0.0, 0.0);
        int c0 = a > b2 ? a : b2;
        for (int c = c0; c < m; ++c) cfmac(acc, A[(size_t)b2 * m + c], A[(size_t)a * m + c]);  // R[a][c] conj(R[b][c])
        G[(size_t)a * m + b2] = acc;
    }
    if (tid == 0) w.gsz[j] = m;
}

// V = Q [W; 0] for the QR-route items, then B_{bond+1} = V^+
template <class T>
__global__ __launch_bounds__(NT) void k_qr_apply(DevState s, DevWork w) {
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (!(d.m < d.n)) return;
    const int m = d.m, n = d.n, tid = threadIdx.x;
    const int k = w.kout[j];
    const double2* A = w.qra + (size_t)j * w.nmax * w.nmax;
    const double2* qt = w.qtau + (size_t)j * w.nmax;
    const int ld = w.vld;
    double2* V = w.V + (size_t)j * w.nmax * ld;
    for (int e = tid; e < (n - m) * k; e += NT) {
        int r = m + e / k, c = e % k;
        V[(size_t)r * ld + c] = mk(0.0, 0.0);
    }
    __syncthreads();
    for (int jj = m - 1; jj >= 0; --jj) {
        const double2 t = qt[jj];
        if (t.x == 0.0 && t.y == 0.0) continue;
        for (int c = tid; c < k; c += NT) {
            double2 acc = V[(size_t)jj * ld + c];
            for (int r = jj + 1; r < n; ++r) cfmac(acc, A[(size_t)r * m + jj], V[(size_t)r * ld + c]);
            acc = cmul(t, acc);
            V[(size_t)jj * ld + c] = csub(V[(size_t)jj * ld + c], acc);
            for (int r = jj + 1; r < n; ++r)
                V[(size_t)r * ld + c] = csub(V[(size_t)r * ld + c], cmul(A[(size_t)r * m + jj], acc));
        }
        __syncthreads();
    }
    if (w.jacobi) return;  // V is refined further; B_{bond+1} is written after the Jacobi sweeps
    T* Br = site_ptr<T>(s, d.b, d.bond + 1);
    for (int e = tid; e < n * k; e += NT) {
        int c = e / n, r = e % n;
        Br[e] = cconv<T>(cconj(V[(size_t)r * ld + c]));
    }
}

// ------------------------------------------------------------------ Householder tridiagonalization
// LAPACK-style lower reduction (reflector H_i = I - tau_i v_i v_i^+, v_i[0] = 1, acting on
// rows i+1..n-1); the off-diagonal of T is made real by the reflector choice, so T is a real
// symmetric tridiagonal matrix (d, e) and H = Q T Q^+ with Q = H_0 H_1 ... H_{n-2}.
#define HETRD_LDS_N 128
template <bool LDS>
__global__ __launch_bounds__(NT) void k_hetrd(DevState s, DevWork w) {
    __shared__ double2 packed_lds[LDS ? (HETRD_LDS_N * (HETRD_LDS_N + 1) / 2) : 1];
    __shared__ double2 vv[512], pp[512];
    __shared__ double red[NT];
    __shared__ double2 redc[NT];
    __shared__ double2 sh_tau, sh_scal, sh_alpha2;
    __shared__ double sh_beta;
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int n = w.gsz[j], tid = threadIdx.x;
    double2* A = LDS ? packed_lds : (w.pscratch + (size_t)j * (w.nmax * (w.nmax + 1) / 2));
    const double2* G = w.gram + (size_t)j * w.nmax * w.nmax;
    double* dd = w.dd + (size_t)j * w.nmax;
    double* ee = w.ee + (size_t)j * w.nmax;
    double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    double2* tau = w.tau + (size_t)j * w.nmax;

    for (int e = tid; e < n * n; e += NT) {
        int r = e / n, c = e % n;
        if (c <= r) A[tri(r, c)] = G[e];
    }
    __syncthreads();

    for (int i = 0; i + 1 < n; ++i) {
        const int len = n - 1 - i;  // length of the reflector
        // ||x||^2 with x = A[i+2 .., i]
        double part = 0.0;
        for (int r = i + 2 + tid; r < n; r += NT) {
            double2 x = A[tri(r, i)];
            part += x.x * x.x + x.y * x.y;
        }
        part = wave_sum(part);
        if ((tid & 63) == 0) red[tid >> 6] = part;
        __syncthreads();
        if (tid == 0) {
            double xn2 = red[0] + red[1] + red[2] + red[3];
            double2 alpha = A[tri(i + 1, i)];
            double2 t, sc;
            double beta;
            if (xn2 == 0.0 && alpha.y == 0.0) {
                t = mk(0.0, 0.0);
                beta = alpha.x;
                sc = mk(1.0, 0.0);
            } else {
                double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                t = mk((beta - alpha.x) / beta, -alpha.y / beta);
                double2 z = mk(alpha.x - beta, alpha.y);  // scal = 1 / z
                double den = z.x * z.x + z.y * z.y;
                sc = mk(z.x / den, -z.y / den);
            }
            sh_tau = t;
            sh_scal = sc;
            sh_beta = beta;
            dd[i] = A[tri(i, i)].x;
            ee[i] = beta;
            tau[i] = t;
        }
        __syncthreads();
        const double2 t = sh_tau, sc = sh_scal;
        for (int r = tid; r < len; r += NT) {
            double2 v = (r == 0) ? mk(1.0, 0.0) : cmul(A[tri(i + 1 + r, i)], sc);
            vv[r] = v;
            refl[(size_t)i * w.nmax + r] = v;
        }
        __syncthreads();
        if (t.x != 0.0 || t.y != 0.0) {
            // p = tau * A22 v  (two threads per row)
            for (int rr = (tid >> 1); rr < len; rr += NT / 2) {
                const int half = tid & 1;
                const int c0 = half ? len / 2 : 0, c1 = half ? len : len / 2;
                const int R = i + 1 + rr;
                double2 acc = mk(0.0, 0.0);
                for (int cc = c0; cc < c1; ++cc) {
                    const int C = i + 1 + cc;
                    double2 a = (cc <= rr) ? A[tri(R, C)] : cconj(A[tri(C, R)]);
                    cfma(acc, a, vv[cc]);
                }
                double ox = __shfl_xor(acc.x, 1), oy = __shfl_xor(acc.y, 1);
                acc.x += ox;
                acc.y += oy;
                if (!half) pp[rr] = cmul(t, acc);
            }
            __syncthreads();
            // alpha2 = -1/2 tau (p^+ v)
            double2 part2 = mk(0.0, 0.0);
            for (int r = tid; r < len; r += NT) cfmac(part2, pp[r], vv[r]);
            part2.x = wave_sum(part2.x);
            part2.y = wave_sum(part2.y);
            if ((tid & 63) == 0) redc[tid >> 6] = part2;
            __syncthreads();
            if (tid == 0) {
                double2 a2 = cmul(t, cadd(cadd(redc[0], redc[1]), cadd(redc[2], redc[3])));
                sh_alpha2 = mk(-0.5 * a2.x, -0.5 * a2.y);
            }
            __syncthreads();
            const double2 a2 = sh_alpha2;
            for (int r = tid; r < len; r += NT) {
                double2 p = pp[r];
                cfma(p, a2, vv[r]);
                pp[r] = p;  // w
            }
            __syncthreads();
            // A22 -= v w^+ + w v^+ (lower triangle)
            for (int rr = tid >> 3; rr < len; rr += NT >> 3) {
                const double2 vr = vv[rr], wr = pp[rr];
                double2* row = A + tri(i + 1 + rr, i + 1);
                for (int cc = tid & 7; cc <= rr; cc += 8) {
                    double2 a = row[cc];
                    double2 u1 = cmulc(pp[cc], vr);  // v_r conj(w_c)
                    double2 u2 = cmulc(vv[cc], wr);  // w_r conj(v_c)
                    a.x -= u1.x + u2.x;
                    a.y -= u1.y + u2.y;
                    row[cc] = a;
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        dd[n - 1] = A[tri(n - 1, n - 1)].x;
        ee[n - 1] = 0.0;
    }
}

// Register-resident reduction for n <= 128 (512 threads, one item per workgroup).  Wave
// (rh, cb) holds rows rh*64 + lane and the 32 columns of block cb, so whole waves drop out once
// their rows or columns are reduced (work ~ n^3/3).  Step i has two block barriers:
//   (B) the partial products A v_i of every column block are in LDS, and the owner of row i+1
//       has published that row as it was before update i;
//   (C) p = tau A v_i and p^+ v_i are final.
// After (C) every wave forms the updated row i+1 and from it the next reflector v_{i+1} (into
// a wave-private, step-parity double-buffered vector), then makes one pass over its tile that
// applies update i and accumulates A v_{i+1} for the next step.  Reflector conventions follow
// LAPACK zhetd2 (lower): H_i = I - tau v v^+, v[i+1] = 1, beta real, so T is real symmetric
// tridiagonal.
#define HR_N 128
#define HR_NT 512
#define HR_NW (HR_NT / 64)
#define HR_CW 32                 // columns per wave tile
#define HR_NCB (HR_N / HR_CW)    // column blocks

// x from lane src - that lane's value where the DPP control selects one, 0 in rows masked off
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}
// sum over the 64 lanes through DPP lane moves (no LDS round trips); every lane gets the total
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
    return readlane_f64(v, 63);
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reflector of the (updated) row i, given as one entry per lane (column lane) for matrices of
// order N = 64, two (columns lane, lane + 64) for N = 128: writes v into this wave's private
// vector vp and returns tau; when wr, also stores d_i, e_i, tau_i and v (into reflrow, the
// reflector's row of the reflector table).
template <int N = HR_N>
__device__ __forceinline__ double2 hr_reflector(int i, int n, int lane, double2 x0, double2 x1, double2* vp,
                                                bool wr, double* dd, double* ee, double2* tau, double2* reflrow) {
    static_assert(N == 64 || N == 128, "one or two columns per lane");
    constexpr bool HI = N > 64;
    const int c0 = lane, c1 = lane + 64;
    double p = 0.0;
    if (c0 >= i + 2 && c0 < n) p += x0.x * x0.x + x0.y * x0.y;
    if (HI && c1 >= i + 2 && c1 < n) p += x1.x * x1.x + x1.y * x1.y;
    p = wave_sum_dpp(p);
    // alpha = conj(row[i+1]) and d_i = row[i] from the lanes that hold them
    const int la = (i + 1) & 63, ld = i & 63;
    const double2 xa = (!HI || (i + 1) < 64) ? x0 : x1, xd = (!HI || i < 64) ? x0 : x1;
    const double2 alpha = mk(readlane_f64(xa.x, la), -readlane_f64(xa.y, la));
    const double di = readlane_f64(xd.x, ld);
    double2 tv, sc;
    double beta;
    if (p == 0.0 && alpha.y == 0.0) {
        tv = mk(0.0, 0.0);
        beta = alpha.x;
        sc = mk(1.0, 0.0);
    } else {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + p);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        // reciprocals: hardware estimate + two Newton steps (a few ulps, shorter chain than
        // the correctly rounded division sequence)
        double ib = __builtin_amdgcn_rcp(beta);
        ib = fma(fma(-beta, ib, 1.0), ib, ib);
        ib = fma(fma(-beta, ib, 1.0), ib, ib);
        tv = mk((beta - alpha.x) * ib, -alpha.y * ib);
        const double2 z = mk(alpha.x - beta, alpha.y);
        const double den = z.x * z.x + z.y * z.y;
        double iden = __builtin_amdgcn_rcp(den);
        iden = fma(fma(-den, iden, 1.0), iden, iden);
        iden = fma(fma(-den, iden, 1.0), iden, iden);
        sc = mk(z.x * iden, -z.y * iden);
    }
    const double2 v0 = (c0 > i && c0 < n) ? ((c0 == i + 1) ? mk(1.0, 0.0) : cmul(cconj(x0), sc)) : mk(0.0, 0.0);
    const double2 v1 = (HI && c1 > i && c1 < n) ? ((c1 == i + 1) ? mk(1.0, 0.0) : cmul(cconj(x1), sc)) : mk(0.0, 0.0);
    wave_fence();  // earlier reads of this buffer by other lanes are done
    vp[c0] = v0;
    if (HI) vp[c1] = v1;
    if (wr) {
        if (c0 > i && c0 < n) reflrow[c0 - i - 1] = v0;
        if (HI && c1 > i && c1 < n) reflrow[c1 - i - 1] = v1;
        if (lane == 0) {
            dd[i] = di;
            ee[i] = beta;
            tau[i] = tv;
        }
    }
    wave_fence();  // the private vector is read by other lanes of this wave
    return tv;
}

// a -= v_r conj(w_c) + w_r conj(v_c)   (the rank-2 update of one matrix entry, 8 FMAs)
__device__ __forceinline__ void hr_rank2(double2& a, double2 vr, double2 wr, double2 vc, double2 wc) {
    a.x = fma(-vr.x, wc.x, a.x);
    a.x = fma(-vr.y, wc.y, a.x);
    a.x = fma(-wr.x, vc.x, a.x);
    a.x = fma(-wr.y, vc.y, a.x);
    a.y = fma(-vr.y, wc.x, a.y);
    a.y = fma(vr.x, wc.y, a.y);
    a.y = fma(-wr.y, vc.x, a.y);
    a.y = fma(wr.x, vc.y, a.y);
}

__global__ __launch_bounds__(HR_NT) void k_hetrd_tile(DevState s, DevWork w) {
    __shared__ double2 vpriv[2][HR_NW][HR_N];
    __shared__ double2 rowold[2][HR_N];
    __shared__ double2 ww[HR_N];
    __shared__ double2 pbuf[HR_NCB * HR_N];
    __shared__ double2 dotp[2];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int n = w.gsz[j], tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int rh = wv / HR_NCB, cb = wv % HR_NCB;
    const int r = rh * 64 + lane, c0 = cb * HR_CW;
    const double2* G = w.gram + (size_t)j * w.nmax * w.nmax;
    double* dd = w.dd + (size_t)j * w.nmax;
    double* ee = w.ee + (size_t)j * w.nmax;
    double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    double2* tau = w.tau + (size_t)j * w.nmax;
    double2 a[HR_CW];
#pragma unroll
    for (int t = 0; t < HR_CW; ++t) {
        const int c = c0 + t;
        double2 v = mk(0.0, 0.0);
        if (r < n && c < n) v = (c <= r) ? G[(size_t)r * n + c] : cconj(G[(size_t)c * n + r]);
        a[t] = v;
    }
    if (n == 1) {
        if (tid == 0) {
            dd[0] = a[0].x;
            ee[0] = 0.0;
        }
        return;
    }
    // every LDS vector starts finite: the branch-free tile pass multiplies stale entries by zero
    for (int e = tid; e < HR_N; e += HR_NT) ww[e] = mk(0.0, 0.0);
    for (int e = tid; e < 2 * HR_NW * HR_N; e += HR_NT) (&vpriv[0][0][0])[e] = mk(0.0, 0.0);
    // reflector 0 from the unreduced row 0, partial A v_0, row 1 published
    if (r == 0) {
#pragma unroll
        for (int t = 0; t < HR_CW; ++t) rowold[0][c0 + t] = a[t];
    }
    __syncthreads();
    double2 tv = hr_reflector(0, n, lane, rowold[0][lane], rowold[0][lane + 64], vpriv[0][wv], wv == 0, dd, ee, tau,
                              refl);
    {
        double2 acc = mk(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < HR_CW; ++t) cfma(acc, a[t], vpriv[0][wv][c0 + t]);
        pbuf[cb * HR_N + r] = acc;
        if (r == 1) {
#pragma unroll
            for (int t = 0; t < HR_CW; ++t) rowold[1][c0 + t] = a[t];
        }
    }
    for (int i = 0; i + 1 < n; ++i) {
        const double2* vc_ = vpriv[i & 1][wv];
        double2* vn_ = vpriv[(i + 1) & 1][wv];
        __syncthreads();  // (B)
        const bool act = !(tv.x == 0.0 && tv.y == 0.0);  // uniform
        if (act && cb == 0) {
            double2 q = mk(0.0, 0.0);
            double2 pr = mk(0.0, 0.0);
            if (r > i && r < n) {
#pragma unroll
                for (int b = 0; b < HR_NCB; ++b) pr = cadd(pr, pbuf[b * HR_N + r]);
                pr = cmul(tv, pr);
                cfmac(q, pr, vc_[r]);
            }
            ww[r] = pr;  // zero outside (i, n)
            q.x = wave_sum_dpp(q.x);
            q.y = wave_sum_dpp(q.y);
            if (lane == 0) dotp[rh] = q;
        }
        __syncthreads();  // (C)
        double2 a2 = mk(0.0, 0.0);
        if (act) {
            const double2 a2t = cmul(tv, cadd(dotp[0], dotp[1]));
            a2 = mk(-0.5 * a2t.x, -0.5 * a2t.y);
        }
        // row i+1 after update i (every wave), then reflector i+1
        double2 x0 = rowold[(i + 1) & 1][lane], x1 = rowold[(i + 1) & 1][lane + 64];
        if (act) {
            const double2 vr = vc_[i + 1];
            double2 wr = ww[i + 1];
            cfma(wr, a2, vr);
            if (lane > i && lane < n) {
                const double2 vc = vc_[lane];
                double2 wc = ww[lane];
                cfma(wc, a2, vc);
                hr_rank2(x0, vr, wr, vc, wc);
            }
            if (lane + 64 > i && lane + 64 < n) {
                const double2 vc = vc_[lane + 64];
                double2 wc = ww[lane + 64];
                cfma(wc, a2, vc);
                hr_rank2(x1, vr, wr, vc, wc);
            }
        }
        const bool more = i + 2 < n;
        double2 tvn = mk(0.0, 0.0);
        if (more) {
            tvn = hr_reflector(i + 1, n, lane, x0, x1, vn_, wv == 0, dd, ee, tau, refl + (size_t)(i + 1) * w.nmax);
        } else if (wv == 0) {
            const double2 xd = (n - 1) < 64 ? x0 : x1;
            const double dl = readlane_f64(xd.x, (n - 1) & 63);
            if (lane == 0) {
                dd[n - 1] = dl;
                ee[n - 1] = 0.0;
            }
        }
        // one pass over the tile: update i, then the partial A v_{i+1} of step i+1.  Branch-free
        // inside (rows outside (i, n) update with v_r = w_r = 0, which leaves them unchanged), so
        // the compiler can batch the LDS reads instead of waiting on each one.
        const bool rows_live = (rh * 64 + 63 > i) && (rh * 64 < n);
        const bool cols_live = (c0 + HR_CW - 1 > i) && (c0 < n);
        double2 acc = mk(0.0, 0.0);
        if (rows_live && cols_live) {  // uniform per wave
            const bool upd = act && r > i && r < n;
            double2 vr = vc_[r], wr = ww[r];
            cfma(wr, a2, vr);
            if (!upd) {
                vr = mk(0.0, 0.0);
                wr = mk(0.0, 0.0);
            }
            double2 acc1 = mk(0.0, 0.0);
#pragma unroll
            for (int t = 0; t < HR_CW; ++t) {
                const double2 vc = vc_[c0 + t];
                double2 wc = ww[c0 + t];
                const double2 vn = vn_[c0 + t];
                cfma(wc, a2, vc);
                hr_rank2(a[t], vr, wr, vc, wc);
                if (t & 1) cfma(acc1, a[t], vn);
                else cfma(acc, a[t], vn);
            }
            acc = cadd(acc, acc1);
        }
        if (more) {
            pbuf[cb * HR_N + r] = acc;
            if (r == i + 2) {
#pragma unroll
                for (int t = 0; t < HR_CW; ++t) rowold[i & 1][c0 + t] = a[t];
            }
        }
        tv = tvn;
    }
}

// MFMA variant for n <= 128 (k_hetrd_mfma<NW, NEXT>: NW waves, one item per workgroup, a matrix of
// order up to 16 NW).  Wave bj owns the block column of columns 16 bj .. 16 bj + 15 over all
// rows, held as NW 16 x 16 blocks in the FP64 MFMA accumulator layout (lane l, element k: row
// l/16 + 4k, column l%16), real and imaginary parts apart.  Per step:
//   p = tau A v for the wave's own 16 indices from the column sums of its blocks (A is
//   Hermitian: p_c = sum_r conj(A_rc) v_r), i.e. per-lane products and a 4-group exchange, so p
//   needs no exchange between waves; p^+ v is summed over waves (barrier 1);
//   w = p - (tau/2)(p^+ v) v is published for all indices (barrier 2);
//   the updated row i+1 and from it reflector i+1 are formed (as in k_hetrd_tile) by every wave
//   (the 8-wave head) or by one wave and published (the 4-wave tail, barrier 3);
//   the rank-2 update A -= v w^+ + w v^+ of each live block is two MFMA 16x16x4 products
//   (real and imaginary part) with [v_r, w_r] as the 16 x 4 operand and [w_c; v_c] as 4 x 16.

// x + (x of lane l ^ 16) and x + (x of lane l ^ 32) in the VALU: swapping a value with a copy of
// itself across half-rows (v_permlane16_swap) or half-waves (v_permlane32_swap) leaves the lane
// and its partner in the two results, so their sum is the pairwise sum (no LDS round trip)
__device__ __forceinline__ double xsum16(double x) {
    const unsigned lo = __double2loint(x), hi = __double2hiint(x);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
__device__ __forceinline__ double xsum32(double x) {
    const unsigned lo = __double2loint(x), hi = __double2hiint(x);
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}

// a_g for the lane's row group g, as a chain of plain selects (v_cndmask) rather than branches
__device__ __forceinline__ double hm_pick(int g, double a0, double a1, double a2, double a3) {
    double r = a0;
    r = g == 1 ? a1 : r;
    r = g == 2 ? a2 : r;
    r = g == 3 ? a3 : r;
    return r;
}

// The reduction in stages.  After reflectors 0 .. K-1 and their updates, the trailing block
// A[K:, K:] is a Hermitian matrix that the remaining reflectors reduce on their own: their rows
// and columns all start at K or later, and the reflector of row K + i of the whole matrix is
// reflector i of the block, entry for entry.  A stage k_hetrd_mfma<NW, NEXT> (NW waves) holds
// the matrix of order min(n, 16 NW) from row and column K0 = max(n - 16 NW, 0); with NEXT > 0 it
// takes the steps down to order NEXT and writes that trailing block back over the Gram matrix,
// in place (row stride n), with NEXT = 0 it reduces its matrix completely.  The stages run as
// 128 -> 64 (8 waves, one item per CU: the order-128 matrix fills half of a CU's registers) and
// 64 -> 1 (4 waves, 122 registers: four items per CU, which hide the latency of each other's
// step chains).  A middle stage 96 -> 64 with 6 waves at two items per CU measured slower than
// taking those steps in the first stage.
template <int NW, int NEXT>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 4 : 2) void k_hetrd_mfma(DevState s, DevWork w) {
    constexpr int N = 16 * NW, NTH = 64 * NW;
    static_assert(NEXT < N && NEXT % 16 == 0, "a stage ends at a smaller order");
    // SH (the four-item-per-CU tail): one wave forms each reflector into a shared vector and a
    // third barrier per step publishes it; the waiting is covered by the other items on the CU,
    // and three of the four waves skip the reflector arithmetic.  The head (one item per CU)
    // keeps a private copy per wave, formed redundantly, and two barriers per step.
    constexpr bool SH = NW == 4;
    constexpr int NVB = SH ? 1 : NW;
    __shared__ double2 vpriv[2][NVB][N];
    __shared__ double2 rowold[2][N];
    __shared__ double2 ww[N];
    __shared__ double2 qpart[NW];
    __shared__ double2 tsh[2];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int nfull = w.gsz[j], tid = threadIdx.x;
    const int K0 = max(nfull - N, 0);                 // first row and column held
    const int n = nfull - K0;                         // order of the held matrix
    if (NEXT > 0 && n <= NEXT) return;                // left whole to the later stages
    const int ilim = NEXT > 0 ? n - NEXT : n - 1;     // steps taken here
    const int wv = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, cl = lane & 15;
    const int C0 = 16 * wv, myc = C0 + cl;
    double2* Gm = w.gram + (size_t)j * w.nmax * w.nmax;
    const double2* G = Gm + (size_t)K0 * nfull + K0;  // row stride nfull
    double* dd = w.dd + (size_t)j * w.nmax + K0;
    double* ee = w.ee + (size_t)j * w.nmax + K0;
    double2* refl = w.refl + ((size_t)j * w.nmax + K0) * w.nmax;
    double2* tau = w.tau + (size_t)j * w.nmax + K0;
    hm_d4 are[NW], aim[NW];
#pragma unroll
    for (int bi = 0; bi < NW; ++bi) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = 16 * bi + g + 4 * k, c = myc;
            double2 v = mk(0.0, 0.0);
            if (r < n && c < n) v = (c <= r) ? G[(size_t)r * nfull + c] : cconj(G[(size_t)c * nfull + r]);
            are[bi][k] = v.x;
            aim[bi][k] = v.y;
        }
    }
    if (n == 1) {
        if (tid == 0) {
            dd[0] = are[0][0];
            ee[0] = 0.0;
        }
        return;
    }
    for (int e = tid; e < N; e += NTH) ww[e] = mk(0.0, 0.0);
    for (int e = tid; e < 2 * NVB * N; e += NTH) (&vpriv[0][0][0])[e] = mk(0.0, 0.0);
    // row 0: block 0, local row 0 (g = 0, k = 0) of every wave
    if (g == 0) rowold[0][myc] = mk(are[0][0], aim[0][0]);
    __syncthreads();
    const int wlast = (n - 1) >> 4;  // owns column n-1: live at every step, writes d, e, tau, v
    const int vw = SH ? 0 : wv;      // this wave's reflector buffer
    const auto hi_half = [&](const double2* row) {
        if constexpr (N > 64) return row[lane + 64];
        else return mk(0.0, 0.0);
    };
    double2 tv = mk(0.0, 0.0);
    if (!SH || wv == wlast) {
        tv = hr_reflector<N>(0, n, lane, rowold[0][lane], hi_half(rowold[0]), vpriv[0][vw], wv == wlast, dd, ee,
                             tau, refl);
        if (SH && lane == 0) tsh[0] = tv;
    }
    if (SH) {
        __syncthreads();
        tv = tsh[0];
    }
    const bool cols_live0 = C0 < n;
    for (int i = 0; i < ilim; ++i) {
        const double2* vc_ = vpriv[i & 1][vw];
        double2* vn_ = vpriv[(i + 1) & 1][vw];
        const bool act = !(tv.x == 0.0 && tv.y == 0.0);  // uniform
        const bool cols_live = cols_live0 && (C0 + 15 > i);
        if (!cols_live) {
            // every column of this wave is reduced: nothing it would compute is read again
            // (later steps use entries > i only); it keeps the barrier count and adds a zero
            // to p^+ v
            if (lane == 0) qpart[wv] = mk(0.0, 0.0);
            __syncthreads();
            __syncthreads();
            if (SH) __syncthreads();
            continue;
        }
        // p_c = tau sum_r conj(A_rc) v_r for the wave's columns c = C0 + cl
        double pr = 0.0, pim = 0.0;
        if (act && cols_live) {
#pragma unroll
            for (int bi = 0; bi < NW; ++bi) {
                if (16 * bi + 15 > i && 16 * bi < n) {  // uniform
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const double2 vr = vc_[16 * bi + g + 4 * k];
                        // conj(a) v
                        pr = fma(are[bi][k], vr.x, pr);
                        pr = fma(aim[bi][k], vr.y, pr);
                        pim = fma(are[bi][k], vr.y, pim);
                        pim = fma(-aim[bi][k], vr.x, pim);
                    }
                }
            }
            // sum over the four row groups (lanes cl, cl+16, cl+32, cl+48)
            pr = xsum32(xsum16(pr));
            pim = xsum32(xsum16(pim));
        }
        const double2 pc = (act && myc > i && myc < n) ? cmul(tv, mk(pr, pim)) : mk(0.0, 0.0);
        if (act) {
            double2 qp = mk(0.0, 0.0);
            if (g == 0) cfmac(qp, pc, vc_[myc]);
            qp.x = wave_sum_dpp(qp.x);
            qp.y = wave_sum_dpp(qp.y);
            if (lane == 0) qpart[wv] = qp;
        }
        // every wave publishes its 16 entries of row i+1 as they are before update i
        {
            const int rl = (i + 1) & 15, bi0 = (i + 1) >> 4;
            if (g == (rl & 3)) {
                const int k0 = rl >> 2;
                double xr = 0.0, xi = 0.0;
#pragma unroll
                for (int bi = 0; bi < NW; ++bi)
                    if (bi == bi0) {
                        xr = hm_pick(k0, are[bi][0], are[bi][1], are[bi][2], are[bi][3]);
                        xi = hm_pick(k0, aim[bi][0], aim[bi][1], aim[bi][2], aim[bi][3]);
                    }
                rowold[(i + 1) & 1][myc] = mk(xr, xi);
            }
        }
        __syncthreads();  // (1)
        double2 a2 = mk(0.0, 0.0);
        if (act) {
            double2 q = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < NW; ++b) q = cadd(q, qpart[b]);
            const double2 a2t = cmul(tv, q);
            a2 = mk(-0.5 * a2t.x, -0.5 * a2t.y);
            if (g == 0) {
                double2 wc = pc;
                cfma(wc, a2, vc_[myc]);
                ww[myc] = wc;  // zero outside (i, n)
            }
        }
        __syncthreads();  // (2)
        double2 tvn = mk(0.0, 0.0);
        if (i + 1 < ilim && (!SH || wv == wlast)) {
            // row i+1 after update i (every wave, or the owner of column n-1 alone), then reflector i+1
            double2 x0 = rowold[(i + 1) & 1][lane], x1 = hi_half(rowold[(i + 1) & 1]);
            if (act) {
                const double2 vr = vc_[i + 1], wr = ww[i + 1];
                if (lane > i && lane < n) hr_rank2(x0, vr, wr, vc_[lane], ww[lane]);
                if constexpr (N > 64)
                    if (lane + 64 > i && lane + 64 < n) hr_rank2(x1, vr, wr, vc_[lane + 64], ww[lane + 64]);
            }
            tvn = hr_reflector<N>(i + 1, n, lane, x0, x1, vn_, wv == wlast, dd, ee, tau,
                                  refl + (size_t)(i + 1) * w.nmax);
            if (SH && lane == 0) tsh[(i + 1) & 1] = tvn;
        } else if (NEXT == 0 && i + 1 >= ilim && wv == wlast) {
            // last diagonal entry: row n-1 after the last update
            double2 xd = rowold[(i + 1) & 1][n - 1];
            if (act) {
                const double2 vr = vc_[n - 1], wr = ww[n - 1];
                hr_rank2(xd, vr, wr, vr, wr);
            }
            if (lane == 0) {
                dd[n - 1] = xd.x;
                ee[n - 1] = 0.0;
            }
        }
        // rank-2 update of the live blocks on MFMA: D += X Y with X = rows of block bi, Y = this column block
        if (act && cols_live) {
            const double2 wc = ww[myc], vc = vc_[myc];
            const double y = hm_pick(g, wc.x, wc.y, vc.x, vc.y);
#pragma unroll
            for (int bi = 0; bi < NW; ++bi) {
                if (16 * bi + 15 > i && 16 * bi < n) {  // uniform
                    const double2 vr = vc_[16 * bi + cl], wr = ww[16 * bi + cl];
                    const double xre = hm_pick(g, -vr.x, -vr.y, -wr.x, -wr.y);
                    const double xim = hm_pick(g, -vr.y, vr.x, -wr.y, wr.x);
                    are[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(xre, y, are[bi], 0, 0, 0);
                    aim[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(xim, y, aim[bi], 0, 0, 0);
                }
            }
        }
        if (SH) {
            __syncthreads();  // (3) reflector i+1 and its tau are published
            if (i + 1 < ilim) tvn = tsh[(i + 1) & 1];
        }
        tv = tvn;
    }
    if (NEXT > 0) {
        // the trailing block after update K-1, both triangles, for the next stage
        const int K = ilim;
        if (myc >= K && myc < n) {
#pragma unroll
            for (int bi = 0; bi < NW; ++bi) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int r = 16 * bi + g + 4 * k;
                    if (r >= K && r < n) Gm[(size_t)(K0 + r) * nfull + K0 + myc] = mk(are[bi][k], aim[bi][k]);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ implicit QL with rotation log
// Tridiagonal QL with implicit Wilkinson-type shifts (one thread per item).  Every
// Givens rotation (i, c, s) is logged; the eigenvector matrix is the ordered product
// Z = G_1 G_2 ... G_N with G acting on columns (i, i+1) as
//   Z[:,i] <- c Z[:,i] - s Z[:,i+1],  Z[:,i+1] <- s Z[:,i] + c Z[:,i+1].
// The working copies of d and e live in LDS (interleaved by lane) when n <= QL_LDS_N.
#define QL_TPB 32
#define QL_LDS_N 128
template <bool LDS>
__device__ __forceinline__ void steqr_item(const DevState& s, const DevWork& w, int j, int lane, double* sdd,
                                           double* see) {
    ItemDims dm;
    if (!item_dims(s, w, j, dm)) return;
    if (w.fb && w.fb[j] != 1) return;  // eigenvectors come from the bisection path
    if (w.fb) atomicAdd(&w.counters[0], 1ull);
    const int n = w.gsz[j];
    double* gd = w.dd + (size_t)j * w.nmax;
    double* ge = w.ee + (size_t)j * w.nmax;
    const int st = LDS ? QL_TPB : 1;
    double* d = LDS ? (sdd + lane) : gd;
    double* e = LDS ? (see + lane) : ge;
    if (LDS)
        for (int i = 0; i < n; ++i) {
            d[i * st] = gd[i];
            e[i * st] = ge[i];
        }
    int* li = w.logi + (size_t)j * w.logcap;
    double2* lcs = w.logcs + (size_t)j * w.logcap;
    const int cap = w.logcap;
    int nr = 0, flag = 0;
    e[(n - 1) * st] = 0.0;
    // absolute deflation floor eps*||T||: the Gram matrix fixes its eigenvalues only to that accuracy,
    // and it lets exactly-zero blocks (product states) deflate at once
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        tnorm = fmax(tnorm, fabs(d[i * st]) + fabs(e[i * st]) + (i > 0 ? fabs(e[(i - 1) * st]) : 0.0));
    const double afloor = DBL_EPSILON * tnorm;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                double em = fabs(e[m * st]);
                double ddm = fabs(d[m * st]) + fabs(d[(m + 1) * st]);
                if (em <= DBL_EPSILON * ddm || em <= afloor) break;
            }
            if (m == l) break;
            if (iter++ >= 60) { flag |= TN_FLAG_NOCONV; break; }
            double g = (d[(l + 1) * st] - d[l * st]) / (2.0 * e[l * st]);
            double r = hypot(g, 1.0);
            g = d[m * st] - d[l * st] + e[l * st] / (g + copysign(r, g));
            double sn = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            double dnext = d[m * st];  // d[i+1], carried in a register along the chase
            double ei_n = e[(m - 1) * st], di_n = d[(m - 1) * st];
            for (int i = m - 1; i >= l; --i) {
                const double ei = ei_n;
                const double di = di_n;
                if (i > l) {  // operands of the next rotation (untouched by this one)
                    ei_n = e[(i - 1) * st];
                    di_n = d[(i - 1) * st];
                }
                double f = sn * ei, bb = c * ei;
                const double r2 = f * f + g * g;
                if (r2 == 0.0) {
                    e[(i + 1) * st] = 0.0;
                    d[(i + 1) * st] = dnext - p;
                    e[m * st] = 0.0;
                    early = true;
                    break;
                }
                // 1/r from the hardware reciprocal square root plus one Newton step
                double rinv = __builtin_amdgcn_rsq(r2);
                rinv = rinv * (1.5 - 0.5 * r2 * rinv * rinv);
                r = r2 * rinv;
                e[(i + 1) * st] = r;
                sn = f * rinv;
                c = g * rinv;
                g = dnext - p;
                r = (di - g) * sn + 2.0 * c * bb;
                p = sn * r;
                d[(i + 1) * st] = g + p;
                g = c * r - bb;
                dnext = di;
                if (nr < cap) {
                    li[nr] = i;
                    lcs[nr] = mk(c, sn);
                } else {
                    flag |= TN_FLAG_LOGFULL;
                }
                ++nr;
            }
            if (early) continue;
            d[l * st] -= p;
            e[l * st] = g;
            e[m * st] = 0.0;
        }
    }
    if (LDS)
        for (int i = 0; i < n; ++i) gd[i] = d[i * st];
    w.nrot[j] = nr < cap ? nr : cap;
    if (flag) atomicOr(w.flags, flag);
}

template <bool LDS>
__global__ __launch_bounds__(QL_TPB) void k_steqr(DevState s, DevWork w) {
    __shared__ double sdd[LDS ? QL_LDS_N * QL_TPB : 1], see[LDS ? QL_LDS_N * QL_TPB : 1];
    steqr_item<LDS>(s, w, blockIdx.x * QL_TPB + threadIdx.x, threadIdx.x, sdd, see);
}

// The logged-QL pass of split mode, which only items holding a degenerate multiplet or a failed
// twisted factorization need (usually none): a small grid scans the chunk.  One workgroup per 32
// items would each wait for a CU slot (64 KB of LDS) behind the other stream's kernels first.
#define QL_FB_BLOCKS 16
__global__ __launch_bounds__(QL_TPB) void k_steqr_fb(DevState s, DevWork w) {
    __shared__ double sdd[QL_LDS_N * QL_TPB], see[QL_LDS_N * QL_TPB];
    for (int j = blockIdx.x * QL_TPB + threadIdx.x; j < w.nitems; j += gridDim.x * QL_TPB) {
        steqr_item<true>(s, w, j, threadIdx.x, sdd, see);
    }
}

// ------------------------------------------------------------------ selection and truncation
// mode 0: Gram eigenvalues (resolution floor rule below), truncate, write Lambda / k / s / weight.
// mode 1: order all r eigenvalues descending into sel (k = r) and nothing else: the full
//         eigenbasis that preconditions the Jacobi refinement.
// mode 2: squared singular values from the Jacobi refinement (resolved to ~eps sigma_0, so the
//         cutoff applies as stated), truncate and write as in mode 0.
__global__ __launch_bounds__(NT) void k_select(DevState s, DevWork w, int mode) {
    __shared__ double lamv[512];
    __shared__ double red[NT];
    __shared__ int redi[NT];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (w.fb && w.fb[j] != 1) return;
    const int n = w.gsz[j], tid = threadIdx.x;
    const double* ev = w.dd + (size_t)j * w.nmax;
    for (int i = tid; i < n; i += NT) lamv[i] = ev[i];
    __syncthreads();
    // max and total (fixed reduction order: deterministic)
    double mx = -1e300, tot = 0.0;
    for (int i = tid; i < n; i += NT) { mx = fmax(mx, lamv[i]); tot += lamv[i]; }
    red[tid] = mx;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) { if (tid < o) red[tid] = fmax(red[tid], red[tid + o]); __syncthreads(); }
    const double lmax = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) { if (tid < o) red[tid] += red[tid + o]; __syncthreads(); }
    const double total = red[0];
    __syncthreads();
    // The Gram route resolves eigenvalues only to ~DBL_EPSILON * lmax (singular values to ~1e-8 sigma_0):
    // a cutoff below that floor cannot be applied faithfully, so every direction is kept (up to chi);
    // discarding a noise-level direction would change the state by up to ~1e-8.
    const double thr = (mode == 0 && s.cutoff2 < 1e-14) ? -1e300 : s.cutoff2 * lmax;
    int cnt = 0;
    for (int i = tid; i < n; i += NT) cnt += (lamv[i] > thr) ? 1 : 0;
    redi[tid] = cnt;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) { if (tid < o) redi[tid] += redi[tid + o]; __syncthreads(); }
    int k = redi[0];
    k = k < s.chi ? k : s.chi;
    k = k < d.m ? k : d.m;
    k = k < n ? k : n;
    if (k < 1) k = 1;
    if (mode == 1) k = n;
    int* sel = w.sel + (size_t)j * w.nmax;
    double kept_part = 0.0;
    for (int i = tid; i < n; i += NT) {
        double li = lamv[i];
        int rk = 0;
        for (int q = 0; q < n; ++q) {
            double lq = lamv[q];
            rk += (lq > li || (lq == li && q < i)) ? 1 : 0;
        }
        if (rk < k) {
            sel[rk] = i;
            kept_part += li;
        }
    }
    __syncthreads();
    if (mode == 1) {
        if (tid == 0) w.kout[j] = k;
        return;
    }
    red[tid] = kept_part;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) { if (tid < o) red[tid] += red[tid + o]; __syncthreads(); }
    double kept = red[0];
    double sv = kept > 0.0 ? sqrt(kept) : 1.0;
    double* lamout = lam_ptr(s, d.b, d.bond);
    for (int r = tid; r < k; r += NT) {
        double li = lamv[sel[r]];
        lamout[r] = li > 0.0 ? sqrt(li) / sv : 0.0;
    }
    if (tid == 0) {
        double wgt = total > 0.0 ? (total - kept) / total : 0.0;
        w.kout[j] = k;
        w.sout[j] = sv;
        w.wout[j] = wgt > 0.0 ? wgt : 0.0;
        if (!(kept == kept) || !(total == total)) atomicOr(w.flags, TN_FLAG_NAN);
    }
}

// ------------------------------------------------------------------ eigenvectors
// Replays the logged rotations in reverse order on the k selected unit vectors (each
// thread owns whole columns, so no synchronization is needed during the replay), then
// applies Q = H_0 ... H_{n-2} (reflectors in reverse order), writes V (n x k, FP64) for
// the split and the new right tensor B_{bond+1} = V^+ (k x n) in storage precision.
#define VECS_LDS_ELEMS 8192
template <class T, bool LDS>
__global__ __launch_bounds__(NT) void k_vecs(DevState s, DevWork w) {
    __shared__ double2 zl[LDS ? VECS_LDS_ELEMS : 1];
    __shared__ int lgi[NT];
    __shared__ double2 lgcs[NT];
    __shared__ double2 vbuf[512];
    __shared__ double2 part[NT];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int n = w.gsz[j], tid = threadIdx.x;
    const int k = w.kout[j];
    const int* sel = w.sel + (size_t)j * w.nmax;
    double2* Z = LDS ? zl : (w.zscratch + (size_t)j * w.nmax * w.vld);
    for (int e = tid; e < n * k; e += NT) {
        int r = e / k, c = e % k;
        Z[e] = mk(r == sel[c] ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // ---- replay rotations, newest first
    const int nr = w.nrot[j];
    const int* li = w.logi + (size_t)j * w.logcap;
    const double2* lcs = w.logcs + (size_t)j * w.logcap;
    for (int hi = nr; hi > 0; hi -= NT) {
        int lo = hi - NT > 0 ? hi - NT : 0;
        int cnt = hi - lo;
        if (tid < cnt) {
            lgi[tid] = li[lo + tid];
            lgcs[tid] = lcs[lo + tid];
        }
        __syncthreads();
        for (int c = tid; c < k; c += NT) {
            for (int q = cnt - 1; q >= 0; --q) {
                const int i = lgi[q];
                const double cc = lgcs[q].x, ss = lgcs[q].y;
                double x = Z[i * k + c].x, y = Z[(i + 1) * k + c].x;
                Z[i * k + c].x = cc * x + ss * y;
                Z[(i + 1) * k + c].x = -ss * x + cc * y;
            }
        }
        __syncthreads();
    }
    // ---- back-transformation by the Householder reflectors
    const double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    const double2* tau = w.tau + (size_t)j * w.nmax;
    // thread layout: group g (4 groups) x column slot cl; columns c = cl, cl+64, ...
    const int g = tid >> 6, cl = tid & 63;
    for (int i = n - 2; i >= 0; --i) {
        const int len = n - 1 - i;
        const double2 t = tau[i];
        if (t.x == 0.0 && t.y == 0.0) continue;  // uniform across the block
        for (int r = tid; r < len; r += NT) vbuf[r] = refl[(size_t)i * w.nmax + r];
        __syncthreads();
        for (int c0 = 0; c0 < k; c0 += 64) {
            const int c = c0 + cl;
            double2 acc = mk(0.0, 0.0);
            if (c < k)
                for (int r = g; r < len; r += 4) cfmac(acc, vbuf[r], Z[(i + 1 + r) * k + c]);
            part[tid] = acc;
            __syncthreads();
            double2 wv = cadd(cadd(part[cl], part[64 + cl]), cadd(part[128 + cl], part[192 + cl]));
            wv = cmul(t, wv);
            if (c < k)
                for (int r = g; r < len; r += 4) {
                    double2 z = Z[(i + 1 + r) * k + c];
                    double2 u = cmul(vbuf[r], wv);
                    z.x -= u.x;
                    z.y -= u.y;
                    Z[(i + 1 + r) * k + c] = z;
                }
            __syncthreads();
        }
    }
    // ---- outputs
    double2* V = w.V + (size_t)j * w.nmax * w.vld;
    T* Br = site_ptr<T>(s, d.b, d.bond + 1);
    for (int e = tid; e < n * k; e += NT) {
        int r = e / k, c = e % k;
        double2 z = Z[e];
        V[(size_t)r * w.vld + c] = z;
    }
    if (!(w.qr_route && d.m < d.n) && !w.jacobi)
        for (int e = tid; e < n * k; e += NT) {
            int c = e / n, r = e % n;  // B_{bond+1}[c][r] = conj(V[r][c])
            Br[e] = cconv<T>(cconj(Z[r * k + c]));
        }
}

// Fast path for n <= 128 and k <= 64: the rotation replay keeps the row that the next
// rotation of the same chase needs in a register (a chase touches rows i, i+1, then i+1, i+2,
// ...), so the dependency chain runs through registers instead of LDS round trips; the real
// eigenvector block Z (n x k doubles, 64 KB) is the only large LDS buffer, and the
// Householder back-transformation runs on Z held in registers (4 row groups x 64 columns).
#define VF_N 128
#define VF_K 64
// Back-transformation of the k eigenvectors of T held in LDS (zr, n x k real, row stride zs) by the
// Householder reflectors: V = Q Z on registers (4 row groups x 64 columns per 256 threads), then
// V (FP64) and B_{bond+1} = V^+ (storage precision) are written.
template <class T>
__device__ __forceinline__ void vf_backtransform(const DevState& s, const DevWork& w, const ItemDims& d, int j, int n,
                                                 int k, const double* zr, int zs, double2* vbuf, double2* part) {
    const int tid = threadIdx.x;
    const int g = tid >> 6, col = tid & 63;
    double2 z[VF_N / 4];
#pragma unroll
    for (int t = 0; t < VF_N / 4; ++t) {
        const int r = g + 4 * t;
        z[t] = (col < k && r < n) ? mk(zr[r * zs + col], 0.0) : mk(0.0, 0.0);
    }
    const double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    const double2* tau = w.tau + (size_t)j * w.nmax;
    // reflector rows stream from memory one step ahead of their use: row i is in registers
    // (cur) while row i+1 is applied, so the global-memory latency overlaps the arithmetic.
    // vbuf holds the reflector zero-padded to full length (vbuf[r] = v_r, 0 for r <= i or r >= n),
    // so the row loops below run without branches and their LDS reads issue together
    double2 cur = (n >= 2 && tid == n - 1) ? refl[(size_t)(n - 2) * w.nmax] : mk(0.0, 0.0);
    double2 tv_cur = n >= 2 ? tau[n - 2] : mk(0.0, 0.0);
    for (int i = n - 2; i >= 0; --i) {
        const double2 tv = tv_cur;
        __syncthreads();  // the previous reflector is no longer read from vbuf / part
        if (tid < VF_N) vbuf[tid] = cur;
        if (i > 0) {
            // next reflector (i-1): entries r = i .. n-1 hold v at offset r - i
            cur = (tid >= i && tid < n) ? refl[(size_t)(i - 1) * w.nmax + (tid - i)] : mk(0.0, 0.0);
            tv_cur = tau[i - 1];
        }
        if (tv.x == 0.0 && tv.y == 0.0) continue;  // uniform across the block
        __syncthreads();
        double2 acc = mk(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < VF_N / 4; ++t) cfmac(acc, vbuf[g + 4 * t], z[t]);
        part[tid] = acc;
        __syncthreads();
        double2 wv = cadd(cadd(part[col], part[64 + col]), cadd(part[128 + col], part[192 + col]));
        wv = cmul(tv, wv);
#pragma unroll
        for (int t = 0; t < VF_N / 4; ++t) {
            const double2 u = cmul(vbuf[g + 4 * t], wv);
            z[t].x -= u.x;
            z[t].y -= u.y;
        }
    }
    double2* V = w.V + (size_t)j * w.nmax * w.vld;
    T* Br = site_ptr<T>(s, d.b, d.bond + 1);
    // the QR route writes B_{bond+1} after expanding V, the Jacobi refinement after its sweeps
    const bool wr_br = !(w.qr_route && d.m < d.n) && !w.jacobi;
    if (col < k) {
#pragma unroll
        for (int t = 0; t < VF_N / 4; ++t) {
            const int r = g + 4 * t;
            if (r < n) {
                V[(size_t)r * w.vld + col] = z[t];
                if (wr_br) Br[(size_t)col * n + r] = cconv<T>(cconj(z[t]));
            }
        }
    }
}

// Blocked back-transformation V = Q Z on the FP64 matrix cores (256 threads, n <= 128, k <= 64).
// Q = H_0 H_1 ... H_{n-2} is applied in blocks of 16 reflectors, the last block first, each in
// the compact WY form H_{a0} ... H_{a0+15} = I - Y T Y^+ (Y: the block's reflectors as columns,
// zero above their unit entries; T upper triangular with T_aa = tau_a and
// T_{0:a, a} = -tau_a T_{0:a, 0:a} (Y_{:, 0:a}^+ y_a), the forward columnwise accumulation), so a
// block costs Z -= Y (T (Y^+ Z)): three 16-wide products instead of 16 rank-1 passes with
// barriers between them.  Complex products are four real 16x16x4 products (real and imaginary
// parts apart).  The row stride BT_LD = 17 of the LDS tiles keeps transposed reads free of bank
// conflicts.
#define BT_LD 17

// tau of reflector a0 + a for a < nr, zero for the padding columns of a short last block
__device__ __forceinline__ double2 tau16v(const double2* tau, int a0, int a, int nr) {
    const double2 t = tau[a0 + min(a, nr - 1)];
    return mk(a < nr ? t.x : 0.0, a < nr ? t.y : 0.0);
}

// T factors of all blocks (they depend only on the reflectors), one wave per block: S = Y^+ Y on
// the matrix cores with both operands read straight from the reflector table (lane l: row
// 16 t + 4 q + l/16 of reflector a0 + l%16 is the A entry conj(.) and the B entry), then lane
// i < 16 forms row i of T from T_ia = -tau_a sum_{m<a} T_im S_ma (T_ii = tau_i, zero left of the
// diagonal), a chain through its own registers.  Block b is stored at tf + 256 b as nr x nr
// (nr: its reflector count), which keeps the table within n^2 entries.  The calling wave is number
// q of nq doing this; blocks go to the waves in snake order of their cost (block b spans
// ntile - b row tiles).  sl: this wave's 16 x 16 scratch.
__device__ __forceinline__ void bt_tfactors(const DevWork& w, int j, int n, int q, int nq, double2* sl,
                                            double2* tf) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, cl = lane & 15;
    const double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    const double2* tau = w.tau + (size_t)j * w.nmax;
    const int nref = n - 1, nblk = (nref + 15) / 16, ntile = (n + 15) >> 4;
    for (int b = 0; b < nblk; ++b) {
        const int rnd = b / nq, pos = b % nq;
        if ((rnd & 1 ? nq - 1 - pos : pos) != q) continue;  // uniform
        const int a0 = 16 * b, nr = min(16, nref - a0);
        const int i = a0 + cl;  // this lane's reflector
        hm_d4 sre = {0.0, 0.0, 0.0, 0.0}, sim = {0.0, 0.0, 0.0, 0.0};
        double2 yc[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const int r = 16 * b + 4 * q4 + g;
            yc[q4] = (cl < nr && r > i && r < n) ? refl[(size_t)i * w.nmax + (r - i - 1)] : mk(0.0, 0.0);
        }
        for (int t = b; t < ntile; ++t) {
            // the next row tile's entries load while this one's products run
            double2 yn[4];
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const int r = 16 * (t + 1) + 4 * q4 + g;
                yn[q4] = (cl < nr && r > i && r < n) ? refl[(size_t)i * w.nmax + (r - i - 1)] : mk(0.0, 0.0);
            }
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const double2 y = yc[q4];
                sre = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, y.x, sre, 0, 0, 0);
                sre = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, y.y, sre, 0, 0, 0);
                sim = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, y.y, sim, 0, 0, 0);
                sim = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.y, y.x, sim, 0, 0, 0);
            }
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) yc[q4] = yn[q4];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) sl[(g + 4 * e) * 16 + cl] = mk(sre[e], sim[e]);
        wave_fence();
        if (lane < 16) {
            double2 trow[16];
            // the reads of column a wait (through an opaque zero offset) for entry a-2: one column
            // of reads ahead of its use, instead of all 120 hoisted to the top and spilled
            int off = 0;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                if (a >= 2) asm volatile("" : "+v"(off) : "v"(trow[a - 2].x));
                double2 acc = mk(0.0, 0.0);
#pragma unroll
                for (int m = 0; m < a; ++m) cfma(acc, trow[m], sl[off + m * 16 + a]);
                const double2 ta = tau16v(tau, a0, a, nr);
                double2 v = cmul(mk(-ta.x, -ta.y), acc);
                // plain selects (a nested choice compiles to divergent branches here)
                v.x = a == lane ? ta.x : v.x;
                v.y = a == lane ? ta.y : v.y;
                v.x = a < lane ? 0.0 : v.x;
                v.y = a < lane ? 0.0 : v.y;
                trow[a] = v;
            }
            if (lane < nr) {
#pragma unroll
                for (int a = 0; a < 16; ++a)
                    if (a < nr) tf[256 * b + lane * nr + a] = trow[a];
            }
        }
        wave_fence();  // sl is rewritten for this wave's next block
    }
}

// Z is held in registers as 16 x 16 tiles in the MFMA accumulator layout (lane l, element e: row
// 16 t + l/16 + 4 e, column 16 wave + l%16).  Element e of a tile is then also the B operand (row
// l/16, column l%16) of the 16x16x4 product over rows 16 t + 4 e .. + 3, so Y^+ Z and T W take
// their right operand from registers; only Y and T come from LDS.  lds: (VF_N + 16) x BT_LD
// entries (Y, then T), inside the caller's Z staging buffer once Z is in registers.
template <class T>
__device__ __forceinline__ void vf_backtransform_mfma(const DevState& s, const DevWork& w, const ItemDims& d, int j,
                                                      int n, int k, const double* zr, int zs, double2* lds,
                                                      const double2* tf) {
    static_assert(NT == 256, "four waves, one 16-column tile of Z each");
    double2* yl = lds;
    double2* tt = yl + VF_N * BT_LD;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, cl = lane & 15;
    const int c = 16 * wv + cl;  // this lane's column of Z
    const int ntile = (n + 15) >> 4;
    hm_d4 zre[VF_N / 16], zim[VF_N / 16];
#pragma unroll
    for (int t = 0; t < VF_N / 16; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * t + g + 4 * e;
            zre[t][e] = (c < k && r < n) ? zr[r * zs + c] : 0.0;
            zim[t][e] = 0.0;
        }
    }
    __syncthreads();  // the staging buffers alias zr
    const double2* refl = w.refl + (size_t)j * w.nmax * w.nmax;
    const int nref = n - 1;  // reflectors 0 .. n-2
    const bool colive = 16 * wv < k;
    // block b's Y entries (thread: rows r = tid % VF_N of reflectors a0 + a, a = tid / VF_N + 2 u)
    // and T entry, loaded into registers one block ahead of their use
    double2 ypf[16 * VF_N / NT], tpf;
    const auto bt_load = [&](int b) {
        const int a0 = 16 * b, nr = min(16, nref - a0);
#pragma unroll
        for (int u = 0; u < 16 * VF_N / NT; ++u) {
            const int e = tid + NT * u, a = e / VF_N, r = e % VF_N, i = a0 + a;
            ypf[u] = (a < nr && r > i && r < n) ? refl[(size_t)i * w.nmax + (r - i - 1)] : mk(0.0, 0.0);
        }
        const int a = tid >> 4, m = tid & 15;
        tpf = (a < nr && m < nr) ? tf[256 * b + a * nr + m] : mk(0.0, 0.0);
    };
    if (nref > 0) bt_load((nref + 15) / 16 - 1);
    for (int b = (nref + 15) / 16 - 1; b >= 0; --b) {
#pragma unroll
        for (int u = 0; u < 16 * VF_N / NT; ++u) {
            const int e = tid + NT * u, a = e / VF_N, r = e % VF_N;
            yl[r * BT_LD + a] = ypf[u];
        }
        tt[(tid >> 4) * BT_LD + (tid & 15)] = tpf;
        __syncthreads();
        if (b > 0) bt_load(b - 1);
        if (colive) {  // uniform per wave
            // W = Y^+ Z (16 x 16, this wave's columns): A = conj(Y[r][l%16]), B = Z[r][c]
            hm_d4 wre = {0.0, 0.0, 0.0, 0.0}, wim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < VF_N / 16; ++t) {
                if (t >= b && t < ntile) {  // uniform
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double2 y = yl[(16 * t + 4 * q + g) * BT_LD + cl];
                        const double zx = zre[t][q], zy = zim[t][q];
                        wre = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, zx, wre, 0, 0, 0);
                        wre = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, zy, wre, 0, 0, 0);
                        wim = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, zy, wim, 0, 0, 0);
                        wim = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.y, zx, wim, 0, 0, 0);
                    }
                }
            }
            // X = T W: A = T[l%16][4 q + l/16], B = W[4 q + l/16][l%16] = element q of W
            hm_d4 xre = {0.0, 0.0, 0.0, 0.0}, xim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 tv = tt[cl * BT_LD + 4 * q + g];
                xre = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.x, wre[q], xre, 0, 0, 0);
                xre = __builtin_amdgcn_mfma_f64_16x16x4f64(-tv.y, wim[q], xre, 0, 0, 0);
                xim = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.x, wim[q], xim, 0, 0, 0);
                xim = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.y, wre[q], xim, 0, 0, 0);
            }
            // Z -= Y X: A = Y[16 t + l%16][4 q + l/16], B = X[4 q + l/16][l%16] = element q of X
#pragma unroll
            for (int t = 0; t < VF_N / 16; ++t) {
                if (t >= b && t < ntile) {  // uniform
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double2 y = yl[(16 * t + cl) * BT_LD + 4 * q + g];
                        zre[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.x, xre[q], zre[t], 0, 0, 0);
                        zre[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, xim[q], zre[t], 0, 0, 0);
                        zim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.x, xim[q], zim[t], 0, 0, 0);
                        zim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y.y, xre[q], zim[t], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();  // Y and T are rewritten for the next block
    }
    double2* V = w.V + (size_t)j * w.nmax * w.vld;
    T* Br = site_ptr<T>(s, d.b, d.bond + 1);
    // the QR route writes B_{bond+1} after expanding V, the Jacobi refinement after its sweeps
    const bool wr_br = !(w.qr_route && d.m < d.n) && !w.jacobi;
    if (c < k) {
#pragma unroll
        for (int t = 0; t < VF_N / 16; ++t) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * t + g + 4 * e;
                if (r < n) {
                    const double2 z = mk(zre[t][e], zim[t][e]);
                    V[(size_t)r * w.vld + c] = z;
                    if (wr_br) Br[(size_t)c * n + r] = cconv<T>(cconj(z));
                }
            }
        }
    }
}

template <class T>
__global__ __launch_bounds__(NT) void k_vecs_fast(DevState s, DevWork w) {
    __shared__ double zr[VF_N * VF_K];
    __shared__ int lgi[NT];
    __shared__ double2 lgcs[NT];
    __shared__ double2 vbuf[VF_N];
    __shared__ double2 part[NT];
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (w.fb && w.fb[j] != 1) return;
    const int n = w.gsz[j], tid = threadIdx.x;
    const int k = w.kout[j];
    const int* sel = w.sel + (size_t)j * w.nmax;
    for (int e = tid; e < n * k; e += NT) zr[e] = (e / k == sel[e % k]) ? 1.0 : 0.0;
    __syncthreads();
    {
        // Replay, newest rotation first; lane c of wave 0 owns column c.  A chase touches rows
        // (i, i+1), (i+1, i+2), ...: the row shared by consecutive rotations stays in a register.
        const int nr = w.nrot[j];
        const int* li = w.logi + (size_t)j * w.logcap;
        const double2* lcs = w.logcs + (size_t)j * w.logcap;
        double xr = 0.0;
        int ci = -1;
        for (int hi = nr; hi > 0; hi -= NT) {
            const int lo = hi - NT > 0 ? hi - NT : 0;
            const int cnt = hi - lo;
            if (tid < cnt) {
                lgi[tid] = li[lo + tid];
                lgcs[tid] = lcs[lo + tid];
            }
            __syncthreads();
            if (tid < k) {
                for (int q = cnt - 1; q >= 0; --q) {
                    const int i = lgi[q];
                    const double cs = lgcs[q].x, sn = lgcs[q].y;
                    double x;
                    if (ci == i) {
                        x = xr;
                    } else {
                        if (ci >= 0) zr[ci * k + tid] = xr;
                        x = zr[i * k + tid];
                    }
                    const double y = zr[(i + 1) * k + tid];
                    zr[i * k + tid] = cs * x + sn * y;
                    xr = -sn * x + cs * y;
                    ci = i + 1;
                }
            }
            __syncthreads();
        }
        if (tid < k && ci >= 0) zr[ci * k + tid] = xr;
    }
    __syncthreads();
    vf_backtransform<T>(s, w, d, j, n, k, zr, k, vbuf, part);
}

// ------------------------------------------------------------------ bisection + twisted factorization (split mode)
// For n <= 128 and chi <= 64 the split path takes the eigenvalues and the k wanted eigenvectors
// of T without a rotation log:
//   k_bisect  lane q of one wavefront finds the q-th largest eigenvalue by bisection on Sturm
//             counts (every lane runs the same recurrence: no divergence); the count above the
//             cutoff, the trace (= sum of all eigenvalues) and the kept sum give k, s, the
//             discarded weight and Lambda as in k_select;
//   k_tvecs   each wanted eigenvector from the twisted factorization of T - lambda I
//             (stationary and progressive LDL^T sweeps, twist where |gamma_r| is smallest), one
//             modified Gram-Schmidt pass in descending order, then the Householder
//             back-transformation.
// Kept eigenvalues closer than 1e-11 lambda_max (a degenerate multiplet, where twisted
// vectors of nearly equal shifts could coincide) take every vector of the item from inverse
// iteration instead, with shifts kept 10 eps ||T|| apart and distinct pseudo-random starts, so
// that a cluster's vectors span its invariant subspace; the Gram-Schmidt pass then makes them
// orthonormal (fb = 3).  A twisted factorization that overflows is redone the same way.  Only
// a tridiagonal that is not finite or has no positive eigenvalue goes to the logged QL path
// (k_steqr, k_select, k_vecs_fast run on those items only): fb = 1.  Two computed eigenvectors
// p, q are orthogonal to about eps lambda_max / |lambda_p - lambda_q|, and the state sees that
// overlap weighted by the singular values of the two directions, sigma_p sigma_q / sigma_0^2 =
// sqrt(lambda_p lambda_q) / lambda_max (the rows of B_{b+1} = V^+ enter every later contraction
// with the weights Lambda_b).  The Gram-Schmidt pass therefore runs when some pair of adjacent
// kept eigenvalues has eps sqrt(lambda_p lambda_q) > 1e-9 |lambda_p - lambda_q| (fb = 2), an
// effect below 1/50 of the complex64 rounding of the stored tensors otherwise; fb = 0.  Close
// pairs at the bottom of a physical spectrum (most bulk bonds of a saturated state hold several
// eigenvalues within 1e-8 lambda_max of each other there) then need no pass.
#define BS_MAXIT 64
#define TV_TIGHT 1e-11
#define TV_ORTH 1e-9

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots of T - x I).  The
// quotient e^2/q uses the hardware reciprocal refined by one Newton step instead of the
// correctly rounded division sequence: a relative error of a few ulps per pivot, the same
// order as the recurrence's own rounding, for about half the instructions (the kernel is
// bound by instruction issue).  |q| >= pivmin >= DBL_MIN keeps the reciprocal finite.
__device__ __forceinline__ int sturm_count(const double* sd, const double* se2, int n, double x, double pivmin) {
    double q = sd[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        double r = __builtin_amdgcn_rcp(q);
        r = fma(fma(-q, r, 1.0), r, r);
        q = fma(-se2[i - 1], r, sd[i] - x);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

__global__ __launch_bounds__(64) void k_bisect(DevState s, DevWork w) {
    __shared__ double sd[VF_N], se2[VF_N];
    const int j = blockIdx.x, lane = threadIdx.x;
    if (j >= w.nitems) return;
    ItemDims dm;
    if (!item_dims(s, w, j, dm)) {
        if (lane == 0) w.fb[j] = 0;
        return;
    }
    const int n = w.gsz[j];
    const double* gd = w.dd + (size_t)j * w.nmax;
    const double* ge = w.ee + (size_t)j * w.nmax;
    double glo = 1e300, ghi = -1e300, tr = 0.0, emax2 = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double di = gd[i];
        const double el = i > 0 ? fabs(ge[i - 1]) : 0.0, er = i + 1 < n ? fabs(ge[i]) : 0.0;
        const double e2 = i + 1 < n ? ge[i] * ge[i] : 0.0;
        sd[i] = di;
        se2[i] = e2;
        glo = fmin(glo, di - el - er);
        ghi = fmax(ghi, di + el + er);
        tr += di;
        emax2 = fmax(emax2, e2);
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    tr = wave_sum(tr);
    emax2 = wave_max(emax2);
    __syncthreads();
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double tol = 4.0 * DBL_EPSILON * tnorm + 2.0 * pivmin;
    const int t = n - 1 - (lane < n ? lane : n - 1);  // ascending index of this lane's eigenvalue
    double lo = glo - tol, hi = ghi + tol;
    for (int it = 0; it < BS_MAXIT; ++it) {
        if (__all(hi - lo <= tol)) break;
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(sd, se2, n, mid, pivmin) <= t) lo = mid;
        else hi = mid;
    }
    const double lam = 0.5 * (lo + hi);
    const double lmax = __shfl(lam, 0);
    int cnt = n;
    if (!(s.cutoff2 < 1e-14)) cnt = n - sturm_count(sd, se2, n, s.cutoff2 * lmax, pivmin);
    int k = cnt < s.chi ? cnt : s.chi;
    k = k < dm.m ? k : dm.m;
    k = k < n ? k : n;
    k = k < VF_K ? k : VF_K;
    if (k < 1) k = 1;
    const double kept = wave_sum(lane < k ? lam : 0.0);
    const double sv = kept > 0.0 ? sqrt(kept) : 1.0;
    const double nxt = __shfl_down(lam, 1);
    const bool tight = lane + 1 < k && !(lam - nxt > TV_TIGHT * lmax);
    const bool close = lane + 1 < k && !(TV_ORTH * (lam - nxt) >= DBL_EPSILON * sqrt(fmax(lam, 0.0) * fmax(nxt, 0.0)));
    const bool bad = !(lmax > 0.0) || !(kept == kept) || !(tr == tr);
    const int fall = bad ? 1 : (__any(tight) ? 3 : (__any(close) ? 2 : 0));
    if (lane < k) {
        lam_ptr(s, dm.b, dm.bond)[lane] = lam > 0.0 ? sqrt(lam) / sv : 0.0;
        w.lsel[(size_t)j * w.nmax + lane] = lam;
    }
    if (lane == 0) {
        const double wgt = tr > 0.0 ? (tr - kept) / tr : 0.0;
        w.kout[j] = k;
        w.sout[j] = sv;
        w.wout[j] = wgt > 0.0 ? wgt : 0.0;
        w.fb[j] = fall;
    }
}

// 1/x from the hardware estimate and two Newton steps: a few ulps, about half the instructions
// of the correctly rounded division on the recurrences' dependency chains (|x| >= pivmin there)
__device__ __forceinline__ double tv_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

// deterministic start entries in [-1, 1): an integer hash of (column, row)
__device__ __forceinline__ double tv_start(int c, int i) {
    unsigned int h = (unsigned int)c * 0x9E3779B1u ^ ((unsigned int)i + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// Eigenvector column c (lane c of wave 0, c < k) of the tridiagonal T (sd, se) by two steps of
// inverse iteration, (T - sigma_c I) x' = x, from a pseudo-random start.  The shifts follow the
// kept eigenvalues in descending order but stay at least 10 eps ||T|| apart: sigma_c =
// min_{p <= c}(lambda_p + p delta) - c delta.  Each solve factors T - sigma_c I = L D L^T top-down
// (pivots kept at least eps ||T|| in size, as inverse iteration allows: a shift on an eigenvalue
// then grows the start by at most 1/(eps ||T||) instead of overflowing; the pivots are kept in the
// item's rotation-log space) and normalizes the result into column c of zr.
__device__ void tv_inverse_iteration(const DevWork& w, int j, int n, int k, int c, const double* sd,
                                     const double* se, double* zr) {
    const double* lsel = w.lsel + (size_t)j * w.nmax;
    const double lam = c < k ? lsel[c] : 0.0;
    double tmax = 0.0;  // max_i |d_i| + |e_{i-1}| + |e_i| >= ||T||
    for (int i = 0; i < n; ++i) tmax = fmax(tmax, fabs(sd[i]) + fabs(se[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0));
    const double delta = 10.0 * DBL_EPSILON * tmax;
    const double pfloor = fmax(DBL_EPSILON * tmax, DBL_MIN);
    // prefix minimum over the lanes of lambda_p + p delta
    double pm = c < k ? lam + c * delta : 1e300;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double v = __shfl_up(pm, o);
        if (c >= o) pm = fmin(pm, v);
    }
    if (c >= k) return;
    const double sig = pm - c * delta;
    double* Dp = reinterpret_cast<double*>(w.logcs + (size_t)j * w.logcap) + (size_t)c * n;
    for (int i = 0; i < n; ++i) zr[i * VF_K + c] = tv_start(c, i);
    for (int it = 0; it < 2; ++it) {
        // forward: D_i and z_i = y_i / D_i with y_i = x_i - (e_{i-1} / D_{i-1}) y_{i-1}
        double dprev = 0.0, yprev = 0.0;
        for (int i = 0; i < n; ++i) {
            double dd = sd[i] - sig;
            double y = zr[i * VF_K + c];
            if (i > 0) {
                const double l = se[i - 1] / dprev;
                dd -= l * se[i - 1];
                y -= l * yprev;
            }
            if (fabs(dd) < pfloor) dd = dd < 0.0 ? -pfloor : pfloor;
            Dp[i] = dd;
            zr[i * VF_K + c] = y / dd;
            dprev = dd;
            yprev = y;
        }
        // backward: x_i = z_i - (e_i / D_i) x_{i+1}, then normalize (by the largest entry first)
        double x = zr[(n - 1) * VF_K + c], amax = fabs(x);
        for (int i = n - 2; i >= 0; --i) {
            x = zr[i * VF_K + c] - (se[i] / Dp[i]) * x;
            zr[i * VF_K + c] = x;
            amax = fmax(amax, fabs(x));
        }
        const double sc = amax > 0.0 ? 1.0 / amax : 0.0;
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            const double v = zr[i * VF_K + c] * sc;
            zr[i * VF_K + c] = v;
            nrm += v * v;
        }
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        for (int i = 0; i < n; ++i) zr[i * VF_K + c] *= inv;
    }
}

template <class T>
__global__ __launch_bounds__(NT, 2) void k_tvecs(DevState s, DevWork w) {
    static_assert((VF_N + 16) * BT_LD * 16 <= VF_N * VF_K * 8, "back-transformation tiles fit in zr");
    __shared__ __align__(16) double zr[VF_N * VF_K];
    __shared__ double sd[VF_N], se[VF_N];
    __shared__ double2 part[NT];
    __shared__ double2 slx[2][256];
    __shared__ int bad;
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    if (w.fb[j] == 1) return;
    const int n = w.gsz[j], tid = threadIdx.x, k = w.kout[j];
    const bool invit = w.fb[j] == 3;
    const double* gd = w.dd + (size_t)j * w.nmax;
    const double* ge = w.ee + (size_t)j * w.nmax;
    for (int i = tid; i < n; i += NT) {
        sd[i] = gd[i];
        se[i] = i + 1 < n ? ge[i] : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    // T factors of the back-transformation blocks (waves 1..3, into the Gram slot, which the
    // Householder reduction no longer needs) while wave 0 forms the eigenvectors of T: a wave
    // takes as long for 16 active lanes as for 64, so one wave carries all k <= 64 columns
    double2* tf = w.gram + (size_t)j * w.nmax * w.nmax;
    const int wv = tid >> 6, ln = tid & 63;
    if (wv > 0) bt_tfactors(w, j, n, wv - 1, NT / 64 - 1, wv == 1 ? part : slx[wv - 2], tf);
    double emax2 = 0.0;
#pragma unroll 8
    for (int i = 0; i + 1 < n; ++i) emax2 = fmax(emax2, se[i] * se[i]);
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    // column c = lane of wave 0: 64 independent recurrences
    const int c = ln;
    if (wv == 0 && c < k && !invit) {
        const double lam = w.lsel[(size_t)j * w.nmax + c];
        // progressive (bottom-up) pivots D-_i of T - lam I, stored in the column
        double dm = sd[n - 1] - lam;
        if (fabs(dm) < pivmin) dm = -pivmin;
        zr[(n - 1) * VF_K + c] = dm;
#pragma unroll 4
        for (int i = n - 2; i >= 0; --i) {
            dm = (sd[i] - lam) - se[i] * se[i] * tv_rcp(dm);
            if (fabs(dm) < pivmin) dm = -pivmin;
            zr[i * VF_K + c] = dm;
        }
        // stationary (top-down) pivots D+_i; twist index r = argmin |gamma_i|, gamma_i = D+_i + D-_i - (d_i - lam)
        double dp = sd[0] - lam;
        if (fabs(dp) < pivmin) dp = -pivmin;
        int r = 0;
        double gbest = fabs(zr[c]);
#pragma unroll 4
        for (int i = 1; i < n; ++i) {
            dp = (sd[i] - lam) - se[i - 1] * se[i - 1] * tv_rcp(dp);
            if (fabs(dp) < pivmin) dp = -pivmin;
            const double gam = fabs(dp + zr[i * VF_K + c] - (sd[i] - lam));
            if (gam < gbest) {
                gbest = gam;
                r = i;
            }
        }
        // D+_i for i < r replace D-_i there (D-_i is needed only below the twist)
        dp = sd[0] - lam;
        if (fabs(dp) < pivmin) dp = -pivmin;
#pragma unroll 4
        for (int i = 0; i < r; ++i) {
            if (i > 0) {
                dp = (sd[i] - lam) - se[i - 1] * se[i - 1] * tv_rcp(dp);
                if (fabs(dp) < pivmin) dp = -pivmin;
            }
            zr[i * VF_K + c] = dp;
        }
        // z_r = 1; below: z_{i+1} = -(e_i / D-_{i+1}) z_i; above: z_i = -(e_i / D+_i) z_{i+1}
        double zi = 1.0, nrm = 1.0;
        zr[r * VF_K + c] = 1.0;
#pragma unroll 4
        for (int i = r; i + 1 < n; ++i) {
            zi = -(se[i] * tv_rcp(zr[(i + 1) * VF_K + c])) * zi;
            zr[(i + 1) * VF_K + c] = zi;
            nrm += zi * zi;
        }
        zi = 1.0;
#pragma unroll 4
        for (int i = r - 1; i >= 0; --i) {
            zi = -(se[i] * tv_rcp(zr[i * VF_K + c])) * zi;
            zr[i * VF_K + c] = zi;
            nrm += zi * zi;
        }
        if (!(nrm < 1e300)) bad = 1;
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < n; ++i) zr[i * VF_K + c] *= inv;
    }
    __syncthreads();
    const bool redo = invit || bad;  // uniform over the workgroup
    if (redo) {
        if (wv == 0) tv_inverse_iteration(w, j, n, k, c, sd, se, zr);
        __syncthreads();
    }
    const bool mgs = redo || w.fb[j] == 2;
    if (tid == 0) {
        if (redo) atomicAdd(&w.counters[0], 1ull);
        if (mgs) atomicAdd(&w.counters[1], 1ull);
    }
    // modified Gram-Schmidt in descending eigenvalue order: column p is final, then removed from p+1..k-1
    const int g = tid >> 6, col = tid & 63;
    for (int p = 0; mgs && p + 1 < k; ++p) {
        double acc = 0.0;
        if (col > p && col < k)
            for (int i = g; i < n; i += 4) acc += zr[i * VF_K + p] * zr[i * VF_K + col];
        part[tid].x = acc;
        __syncthreads();
        const double dot = part[col].x + part[64 + col].x + part[128 + col].x + part[192 + col].x;
        double sq = 0.0;
        if (col > p && col < k)
            for (int i = g; i < n; i += 4) {
                const double v = zr[i * VF_K + col] - dot * zr[i * VF_K + p];
                zr[i * VF_K + col] = v;
                sq += v * v;
            }
        __syncthreads();
        part[tid].x = sq;
        __syncthreads();
        if (col > p && col < k) {
            const double inv = 1.0 / sqrt(part[col].x + part[64 + col].x + part[128 + col].x + part[192 + col].x);
            for (int i = g; i < n; i += 4) zr[i * VF_K + col] *= inv;
        }
        __syncthreads();
    }
    vf_backtransform_mfma<T>(s, w, d, j, n, k, zr, VF_K, reinterpret_cast<double2*>(zr), tf);
}

// ------------------------------------------------------------------ Hastings split
// B_bond = Theta~ V / s on the FP64 matrix cores in both precisions: V is the FP64 eigenvector
// matrix and Theta~ the FP64 workspace copy, so the only rounding of the split is the final
// store.  FP32 products here would round V and Theta~ at every update, a per-update error
// several times that of the store.  The launch bound asks for three workgroups per CU; the
// compiler then keeps the accumulators in 104 VGPRs (instead of 106 + 64 AGPRs) and four fit per
// CU, a third less time than at two.
template <class T>
__global__ __launch_bounds__(NT, 3) void k_split(DevState s, DevWork w, int tiles_n, double* glog, double* gwt) {
    __shared__ double2 As[8 * 64], Bs[8 * 64];
    ItemDims d;
    const int j = blockIdx.y;
    if (!item_dims(s, w, j, d)) return;
    const int k = w.kout[j];
    const double sv = w.sout[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.dims[(size_t)d.b * (s.L + 1) + d.bond + 1] = k;
        const size_t g = (size_t)d.b * w.nb + (d.bond - w.parity) / 2;  // per instance and bond position
        glog[g] = log(sv);
        gwt[g] = w.wout[j];
    }
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= d.m || tn * 64 >= k) return;
    typedef typename real_of<T>::type R;
    const double2* th = reinterpret_cast<const double2*>(w.theta) + (size_t)j * w.theta_stride;
    const double2* V = w.V + (size_t)j * w.nmax * w.vld;
    T* Bl = site_ptr<T>(s, d.b, d.bond);
    const int n = d.n, chi = w.vld;
    const double inv = 1.0 / sv;
    if (w.rmove) {
        // centre moves right: B_bond = Theta~ V diag(1/S) (left isometry), B_{bond+1} <- diag(Lambda) V^+
        const double* lam = lam_ptr(s, d.b, d.bond);
        if (blockIdx.x == 0) {
            T* Br = site_ptr<T>(s, d.b, d.bond + 1);
            for (int e = threadIdx.x; e < k * n; e += NT) Br[e] = cscale(Br[e], (R)lam[e / n]);
        }
        block_gemm<double2, true, true, 8>(
            d.m, k, n, tm * 64, tn * 64,
            [&](int r, int q) { return th[(size_t)r * n + q]; },
            [&](int q, int c) { return V[(size_t)q * chi + c]; },
            [&](int r, int c, double2 v) {
                const double sc = lam[c] > 0.0 ? 1.0 / (lam[c] * sv) : 0.0;
                Bl[(size_t)r * k + c] = cconv<T>(cscale(v, sc));
            }, As, Bs);
        return;
    }
    block_gemm<double2, true, true, 8>(
        d.m, k, n, tm * 64, tn * 64,
        [&](int r, int q) { return th[(size_t)r * n + q]; },
        [&](int q, int c) { return V[(size_t)q * chi + c]; },
        [&](int r, int c, double2 v) { Bl[(size_t)r * k + c] = cconv<T>(cscale(v, inv)); }, As, Bs);
}

// ------------------------------------------------------------------ FP64 mode: one-sided Jacobi refinement
// The Gram eigenvalues carry an absolute error of ~eps * sigma_0^2, so singular values below
// ~sqrt(eps) sigma_0 (~1e-8 sigma_0) are not resolved, and a truncation among them would be
// decided by rounding.  In FP64 mode every Gram eigenvector is formed (V, n x r), and the columns
// of Y = Theta~ V are made orthogonal in the Lambda_{bond-1}^2-weighted inner product by one-sided
// (Hestenes) Jacobi rotations applied to Y and V alike.  The singular values of Theta are then
// the weighted column norms of Y, resolved to ~eps sigma_0, and Y itself is Theta~ V for the
// Hastings split.  The Gram basis leaves only clusters of nearly equal small singular values to
// rotate, so a few sweeps converge.
__global__ __launch_bounds__(NT) void k_jac_y(DevState s, DevWork w, int tiles_n) {
    __shared__ double2 As[8 * 64], Bs[8 * 64];
    ItemDims d;
    const int j = blockIdx.y;
    if (!item_dims(s, w, j, d)) return;
    const int r = w.kout[j];
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= d.m || tn * 64 >= r) return;
    const double2* th = reinterpret_cast<const double2*>(w.theta) + (size_t)j * w.theta_stride;
    const double2* V = w.V + (size_t)j * w.nmax * w.vld;
    double2* Y = w.Y + (size_t)j * w.ysz;
    const int n = d.n, ld = w.vld, ldy = w.ldy;
    block_gemm<double2, true, true, 8>(
        d.m, r, n, tm * 64, tn * 64,
        [&](int i, int q) { return th[(size_t)i * n + q]; },
        [&](int q, int c) { return V[(size_t)q * ld + c]; },
        [&](int i, int c, double2 v) { Y[(size_t)c * ldy + i] = v; }, As, Bs);
}

#define JAC_NT 512
#define JAC_SWEEPS 30
// One workgroup per item.  Sweeps follow a round-robin tournament over the r columns (column 0
// fixed, the others rotating; one bye when r is odd): each round is a set of disjoint pairs, one
// wavefront per pair, so rounds need only a barrier between them.  A pair is rotated when its
// weighted cosine exceeds eps*sqrt(m) and both columns are above the rounding floor
// (eps^2 * sum of all squared norms); the sweeps stop when a sweep rotates nothing.
__global__ __launch_bounds__(JAC_NT) void k_jacobi(DevState s, DevWork w) {
    __shared__ double wt[1024];  // row weights: m = d_l chi_l <= 1024
    __shared__ double redv[JAC_NT / 64];
    __shared__ int rotated;
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int m = d.m, n = d.n, r = w.kout[j], tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int NW = JAC_NT / 64;
    const double* lamL = (d.bond > 0 && !w.unitw) ? lam_ptr(s, d.b, d.bond - 1) : nullptr;
    for (int i = tid; i < m; i += JAC_NT) {
        const double l = lamL ? lamL[i / d.dl] : 1.0;
        wt[i] = l * l;
    }
    __syncthreads();
    double2* Y = w.Y + (size_t)j * w.ysz;
    double2* V = w.V + (size_t)j * w.nmax * w.vld;
    const int ldy = w.ldy, ld = w.vld;
    double p = 0.0;
    for (int c = wv; c < r; c += NW)
        for (int i = lane; i < m; i += 64) {
            const double2 y = Y[(size_t)c * ldy + i];
            p += wt[i] * (y.x * y.x + y.y * y.y);
        }
    p = wave_sum(p);
    if (lane == 0) redv[wv] = p;
    __syncthreads();
    double total = 0.0;
    for (int q = 0; q < NW; ++q) total += redv[q];
    // A pair (p, q) is rotated when its coupling g = |y_p^+ W y_q| exceeds both the relative
    // tolerance eps sqrt(m) |y_p| |y_q| and an absolute floor (m eps)^2 sum sigma^2.  The mixing
    // that the Gram basis leaves between directions is about eps sigma_0^2, far above the floor,
    // so it is always removed; what a rotation leaves behind in floating point is below it, so
    // the sweeps end.  Without the floor, pairs involving columns near the rounding level of
    // Y = Theta~ V (absolute errors about eps sigma_0) keep re-triggering the relative test.
    // A coupling left below the floor changes the state by about g / sigma_max.  Columns below
    // eps of the total are numerically zero and never rotated.
    const double floor2 = DBL_EPSILON * DBL_EPSILON * total;
    const double gfloor = ((double)m * DBL_EPSILON) * ((double)m * DBL_EPSILON) * total;
    const double tol = DBL_EPSILON * sqrt((double)m);
    const int R = r + (r & 1);
    int sweep = 0;
    for (; sweep < JAC_SWEEPS; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        int any = 0;
        for (int t = 0; t < R - 1; ++t) {
            for (int pi = wv; pi < R / 2; pi += NW) {
                int a, b;
                if (pi == 0) {
                    a = 0;
                    b = 1 + t % (R - 1);
                } else {
                    a = 1 + (t + pi) % (R - 1);
                    b = 1 + (t - pi + (R - 1)) % (R - 1);
                }
                if (a > b) { const int x = a; a = b; b = x; }
                if (b >= r) continue;  // bye
                double2* yp = Y + (size_t)a * ldy;
                double2* yq = Y + (size_t)b * ldy;
                double app = 0.0, aqq = 0.0, cx = 0.0, cy = 0.0;
                for (int i = lane; i < m; i += 64) {
                    const double2 u = yp[i], v = yq[i];
                    const double ww = wt[i];
                    app += ww * (u.x * u.x + u.y * u.y);
                    aqq += ww * (v.x * v.x + v.y * v.y);
                    cx += ww * (u.x * v.x + u.y * v.y);
                    cy += ww * (u.x * v.y - u.y * v.x);
                }
                app = wave_sum(app);
                aqq = wave_sum(aqq);
                cx = wave_sum(cx);
                cy = wave_sum(cy);
                const double g = sqrt(cx * cx + cy * cy);
                if (!(app > floor2 && aqq > floor2) || !(g > tol * sqrt(app * aqq)) || !(g > gfloor)) continue;
                // rotate (p, q~ = conj(ph) q), ph = c/|c|, by the real Jacobi angle of [[app, g], [g, aqq]]
                const double zeta = (aqq - app) / (2.0 * g);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                const double2 ph = mk(cx / g, cy / g), phc = mk(cx / g, -cy / g);
                for (int i = lane; i < m; i += 64) {
                    const double2 u = yp[i], v = yq[i];
                    const double2 cv = cmul(phc, v), pu = cmul(ph, u);
                    yp[i] = mk(cs * u.x - sn * cv.x, cs * u.y - sn * cv.y);
                    yq[i] = mk(sn * pu.x + cs * v.x, sn * pu.y + cs * v.y);
                }
                for (int q = lane; q < n; q += 64) {
                    const double2 u = V[(size_t)q * ld + a], v = V[(size_t)q * ld + b];
                    const double2 cv = cmul(phc, v), pu = cmul(ph, u);
                    V[(size_t)q * ld + a] = mk(cs * u.x - sn * cv.x, cs * u.y - sn * cv.y);
                    V[(size_t)q * ld + b] = mk(sn * pu.x + cs * v.x, sn * pu.y + cs * v.y);
                }
                any = 1;
            }
            __syncthreads();
        }
        if (any) rotated = 1;
        __syncthreads();
        const int done = !rotated;
        __syncthreads();
        if (done) break;
    }
    if (sweep == JAC_SWEEPS && tid == 0) atomicOr(w.flags, TN_FLAG_JACOBI);
    // squared singular values = weighted column norms (into the eigenvalue slot for k_select)
    for (int c = wv; c < r; c += NW) {
        double q2 = 0.0;
        for (int i = lane; i < m; i += 64) {
            const double2 y = Y[(size_t)c * ldy + i];
            q2 += wt[i] * (y.x * y.x + y.y * y.y);
        }
        q2 = wave_sum(q2);
        if (lane == 0) w.dd[(size_t)j * w.nmax + c] = q2;
    }
}

// B_bond = Y[:, sel] / s (= Theta~ V / s), B_{bond+1} = V[:, sel]^+, dims, log s and weight per item
template <class T>
__global__ __launch_bounds__(NT) void k_jac_store(DevState s, DevWork w, double* glog, double* gwt) {
    ItemDims d;
    const int j = blockIdx.x;
    if (!item_dims(s, w, j, d)) return;
    const int k = w.kout[j], m = d.m, n = d.n, tid = threadIdx.x;
    const double sv = w.sout[j];
    if (tid == 0) {
        s.dims[(size_t)d.b * (s.L + 1) + d.bond + 1] = k;
        const size_t g = (size_t)d.b * w.nb + (d.bond - w.parity) / 2;  // per instance and bond position
        glog[g] = log(sv);
        gwt[g] = w.wout[j];
    }
    const int* sel = w.sel + (size_t)j * w.nmax;
    const double2* Y = w.Y + (size_t)j * w.ysz;
    const double2* V = w.V + (size_t)j * w.nmax * w.vld;
    T* Bl = site_ptr<T>(s, d.b, d.bond);
    T* Br = site_ptr<T>(s, d.b, d.bond + 1);
    const double inv = 1.0 / sv;
    // centre moving right (sequential sweep): B_bond = Y diag(1/S), B_{bond+1} = diag(Lambda) V^+
    const double* lam = w.rmove ? lam_ptr(s, d.b, d.bond) : nullptr;
    for (int e = tid; e < m * k; e += NT) {
        const int i = e / k, c = e % k;
        const double sc = lam ? (lam[c] > 0.0 ? 1.0 / (lam[c] * sv) : 0.0) : inv;
        Bl[e] = cconv<T>(cscale(Y[(size_t)sel[c] * w.ldy + i], sc));
    }
    for (int e = tid; e < k * n; e += NT) {
        const int c = e / n, q = e % n;
        const double2 v = cconj(V[(size_t)q * w.vld + sel[c]]);
        Br[e] = cconv<T>(lam ? cscale(v, lam[c]) : v);
    }
}

// per instance: add the log-norms and discarded weights of its items (fixed order)
__global__ void k_reduce_items(DevState s, int nb, int parity, const unsigned char* mask,
                               const double* glog, const double* gwt) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.B) return;
    if (mask && mask[b]) return;
    double lg = 0.0, wt = 0.0;
    for (int t = 0; t < nb; ++t) {
        lg += glog[(size_t)b * nb + t];
        wt += gwt[(size_t)b * nb + t];
    }
    s.lognorm[b] += lg;
    s.trunc[b] += wt;
}

// ------------------------------------------------------------------ host launchers
#include "launch.h"

// One chunk of a layer in five phases (all in stream order on `st`):
//   0 light: Theta, gate, Gram (+ QR of wide items)      1 heavy: Householder reduction
//   2 light: eigenvalues (bisection / QL + selection)     3 heavy: eigenvectors (+ QR apply)
//   4 light: split and the rest
// Heavy phases hold one or two workgroups per compute unit through their register use; a caller
// that runs two chunks on two streams can order the heavy phases of both so that light phases of
// one chunk share the compute units with a heavy phase of the other.
// weighted Gram matrix (and, on the QR route, the wide-Theta factorization that replaces it)
// Theta~ (with the gate unless w.skip_gate) into the workspace, contracted in operand type TC
template <class T, class TC>
static void launch_theta(const DevState& s, const DevWork& w, hipStream_t st) {
    const int tm = (w.mmax + 63) / 64, tn = (w.nmax + 63) / 64;
    if (w.skip_gate) {
        hipLaunchKernelGGL((k_theta<T, TC>), dim3(tm * tn, w.nitems), dim3(NT), 0, st, s, w, tn);
        return;
    }
    // virtual column tiles: 64/d_r values of c per tile, for the largest d_r
    const int tv = (s.chi * s.dmax + 63) / 64;
    if (s.dmax == 2)
        hipLaunchKernelGGL((k_theta_gate<T, TC, 4>), dim3(tm * tv, w.nitems), dim3(NT), 0, st, s, w, tv);
    else
        hipLaunchKernelGGL((k_theta_gate<T, TC, 16>), dim3(tm * tv, w.nitems), dim3(NT), 0, st, s, w, tv);
}

template <class T>
static void launch_gram(const DevState& s, const DevWork& w, hipStream_t st) {
    if (w.nmax > 64 && w.nmax <= 128) {
        // (for n <= 64 only the tile rows 0..3 exist and the matrix-core kernel measured slower)
        hipLaunchKernelGGL(k_gram_mfma<T>, dim3(w.nitems), dim3(NT), 0, st, s, w);
    } else {
        const int tn = (w.nmax + 63) / 64;
        hipLaunchKernelGGL(k_gram<T>, dim3(tn * tn, w.nitems), dim3(NT), 0, st, s, w, tn);
    }
    if (w.qr_route) hipLaunchKernelGGL(k_qr_wide, dim3(w.nitems), dim3(NT), 0, st, s, w);
}

// stages of the MFMA Householder reduction, n <= 128 (a stage leaves smaller items untouched)
static void launch_hetrd_mfma(const DevState& s, const DevWork& w, hipStream_t st) {
    if (w.nmax > 64) hipLaunchKernelGGL((k_hetrd_mfma<8, 64>), dim3(w.nitems), dim3(512), 0, st, s, w);
    hipLaunchKernelGGL((k_hetrd_mfma<4, 0>), dim3(w.nitems), dim3(256), 0, st, s, w);
}

template <class T>
static void launch_layer_phase_t(const DevState& s, const DevWork& w, int phase, hipStream_t st, Prof* prof,
                                 double* glog, double* gwt) {
    const int tm = (w.mmax + 63) / 64, tn = (w.nmax + 63) / 64;
    const int tkn = (s.chi + 63) / 64;
    switch (phase) {
    case 0:
        prof_begin(prof, TN_K_THETA, st);
        if (w.theta64) launch_theta<T, double2>(s, w, st);
        else launch_theta<T, T>(s, w, st);
        prof_end(prof, TN_K_THETA, st);
        prof_begin(prof, TN_K_GRAM, st);
        launch_gram<double2>(s, w, st);
        prof_end(prof, TN_K_GRAM, st);
        return;
    case 1:
        prof_begin(prof, TN_K_HETRD, st);
        if (w.nmax <= HR_N && w.hvar == 1)
            hipLaunchKernelGGL(k_hetrd_tile, dim3(w.nitems), dim3(HR_NT), 0, st, s, w);
        else if (w.nmax <= HR_N)
            launch_hetrd_mfma(s, w, st);
        else if (w.nmax <= HETRD_LDS_N)
            hipLaunchKernelGGL(k_hetrd<true>, dim3(w.nitems), dim3(NT), 0, st, s, w);
        else
            hipLaunchKernelGGL(k_hetrd<false>, dim3(w.nitems), dim3(NT), 0, st, s, w);
        prof_end(prof, TN_K_HETRD, st);
        return;
    case 2:
        prof_begin(prof, TN_K_STEQR, st);
        if (w.fb) {
            // split mode, n <= 128, chi <= 64: bisection + twisted factorization; the logged QL
            // path runs only on the items that k_bisect or k_tvecs hand over
            hipLaunchKernelGGL(k_bisect, dim3(w.nitems), dim3(64), 0, st, s, w);
        } else {
            if (w.nmax <= QL_LDS_N)
                hipLaunchKernelGGL(k_steqr<true>, dim3((w.nitems + QL_TPB - 1) / QL_TPB), dim3(QL_TPB), 0, st, s, w);
            else
                hipLaunchKernelGGL(k_steqr<false>, dim3((w.nitems + QL_TPB - 1) / QL_TPB), dim3(QL_TPB), 0, st, s, w);
            hipLaunchKernelGGL(k_select, dim3(w.nitems), dim3(NT), 0, st, s, w, w.jacobi ? 1 : 0);
        }
        prof_end(prof, TN_K_STEQR, st);
        return;
    case 3:
        prof_begin(prof, TN_K_VECS, st);
        if (w.fb) {
            hipLaunchKernelGGL(k_tvecs<T>, dim3(w.nitems), dim3(NT), 0, st, s, w);
        } else {
            if (w.nmax <= VF_N && w.vld <= VF_K)
                hipLaunchKernelGGL(k_vecs_fast<T>, dim3(w.nitems), dim3(NT), 0, st, s, w);
            else if ((size_t)w.nmax * w.vld <= VECS_LDS_ELEMS)
                hipLaunchKernelGGL((k_vecs<T, true>), dim3(w.nitems), dim3(NT), 0, st, s, w);
            else
                hipLaunchKernelGGL((k_vecs<T, false>), dim3(w.nitems), dim3(NT), 0, st, s, w);
            if (w.qr_route) hipLaunchKernelGGL(k_qr_apply<T>, dim3(w.nitems), dim3(NT), 0, st, s, w);
        }
        prof_end(prof, TN_K_VECS, st);
        return;
    default:
        if (w.fb) {
            const int nb = (w.nitems + QL_TPB - 1) / QL_TPB;
            hipLaunchKernelGGL(k_steqr_fb, dim3(nb < QL_FB_BLOCKS ? nb : QL_FB_BLOCKS), dim3(QL_TPB), 0, st, s, w);
            hipLaunchKernelGGL(k_select, dim3(w.nitems), dim3(NT), 0, st, s, w, 0);
            hipLaunchKernelGGL(k_vecs_fast<T>, dim3(w.nitems), dim3(NT), 0, st, s, w);
        }
        prof_begin(prof, TN_K_SPLIT, st);
        if (w.jacobi) {
            const int tr = (w.nmax + 63) / 64;
            hipLaunchKernelGGL(k_jac_y, dim3(tm * tr, w.nitems), dim3(NT), 0, st, s, w, tr);
            hipLaunchKernelGGL(k_jacobi, dim3(w.nitems), dim3(JAC_NT), 0, st, s, w);
            hipLaunchKernelGGL(k_select, dim3(w.nitems), dim3(NT), 0, st, s, w, 2);
            hipLaunchKernelGGL(k_jac_store<T>, dim3(w.nitems), dim3(NT), 0, st, s, w, glog, gwt);
        } else {
            hipLaunchKernelGGL(k_split<T>, dim3(tm * tkn, w.nitems), dim3(NT), 0, st, s, w, tkn, glog, gwt);
        }
        prof_end(prof, TN_K_SPLIT, st);
        return;
    }
}

void launch_layer_phase(int prec, const DevState& s, const DevWork& w, int phase, hipStream_t st, Prof* prof,
                        double* glog, double* gwt) {
    if (prec == 0)
        launch_layer_phase_t<double2>(s, w, phase, st, prof, glog, gwt);
    else
        launch_layer_phase_t<float2>(s, w, phase, st, prof, glog, gwt);
}

void launch_layer_chunk(int prec, const DevState& s, const DevWork& w, hipStream_t st, Prof* prof,
                        double* glog, double* gwt) {
    for (int ph = 0; ph < 5; ++ph) launch_layer_phase(prec, s, w, ph, st, prof, glog, gwt);
}

template <class T>
static void launch_update_prefix_t(const DevState& s, const DevWork& w, hipStream_t st) {
    if (w.theta64) launch_theta<T, double2>(s, w, st);
    else launch_theta<T, T>(s, w, st);
    launch_gram<double2>(s, w, st);
}

void launch_update_prefix(int prec, const DevState& s, const DevWork& w, hipStream_t st) {
    if (prec == 0)
        launch_update_prefix_t<double2>(s, w, st);
    else
        launch_update_prefix_t<float2>(s, w, st);
}

void launch_hetrd_variant(const DevState& s, const DevWork& w, int variant, hipStream_t st) {
    if (variant == 1)
        hipLaunchKernelGGL(k_hetrd_tile, dim3(w.nitems), dim3(HR_NT), 0, st, s, w);
    else
        launch_hetrd_mfma(s, w, st);
}

void launch_reduce_items(const DevState& s, int nb, int parity, const unsigned char* mask, const double* glog,
                         const double* gwt, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_items, dim3((s.B + 127) / 128), dim3(128), 0, st, s, nb, parity, mask, glog, gwt);
}
