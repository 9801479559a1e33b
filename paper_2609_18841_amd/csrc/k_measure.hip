// Measurement sweep C_ij = <c_i^+ c_j> (Sec. 2.1) by exact, gauge-independent contraction.
//
// Pure states and purified X (physical index p = n*dk + k, operators act on n only):
//   right environments  R_j[a'][a] = sum_p conj(B_j^p) R_{j+1} B_j^p^T       (R_L = 1)
//   left  environment   E_j        = sum_p B_j^p^+ E_{j-1} B_j^p               (E_{-1} = 1)
//   open strings X_i    created at site i with s+ from E_{i-1}, carried with F = (-1)^n,
//   closed at every j > i with s- against R_{j+1}: c_i^+ c_j = s+_i (prod F) s-_j.
// Per site j all open strings share B_j, so each step is a batch of small GEMMs
//   Y = X . B_j   (chi_l x d chi_r),   W = conj(B_j) . R_{j+1}   (chi_l d x chi_r),
//   C_ij = sum <Y[(n=1,k)], W[(n'=0,k)]> (FP64 accumulation),   X <- sum_p s_p B_j^p^+ Y^p.
// Vectorized density matrices use the local trace vectors t_O[m = n*2 + n'] = O[n', n]
// and only vector-matrix products (Sec. 3.1).
#include "common.h"
#include "gemm.h"
#include "launch.h"

#define NT 256

struct SiteDims { int chil, chir, d, dk; };
__device__ __forceinline__ SiteDims site_dims(const DevState& s, int b, int j) {
    SiteDims r;
    r.chil = bond_dim(s, b, j);
    r.chir = bond_dim(s, b, j + 1);
    r.d = s.dsite[j];
    r.dk = r.d / 2;
    return r;
}

__host__ __device__ __forceinline__ size_t cc(int chi) { return (size_t)chi * chi; }

// ---------------------------------------------------------------- right environments
// U[(a,p)][c'] = sum_c B[(a,p)][c] R_{j+1}[c'][c]
template <class T>
__global__ __launch_bounds__(NT) void k_env_right_a(DevState s, MeasWork mw, int j, int tiles_n) {
    __shared__ T As[8 * 64], Bs[8 * 64];
    const int bi = blockIdx.y, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int M = sd.chil * sd.d, N = sd.chir, K = sd.chir;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= M || tn * 64 >= N) return;
    const T* P = site_ptr<T>(s, b, j);
    const T* R = reinterpret_cast<const T*>(mw.R) + ((size_t)(j + 1) * mw.nbm + bi) * cc(s.chi);
    T* U = reinterpret_cast<T*>(mw.W) + (size_t)bi * s.chi * s.dmax * s.chi;
    block_gemm<T, true, false, 8>(
        M, N, K, tm * 64, tn * 64,
        [&](int r, int c) { return P[(size_t)r * K + c]; },
        [&](int c, int cp) { return R[(size_t)cp * K + c]; },
        [&](int r, int cp, double2 v) { U[(size_t)r * N + cp] = cconv<T>(v); }, As, Bs);
}

// R_j[a'][a] = sum_{(p,c')} conj(B[a'][(p,c')]) U[a][(p,c')]
template <class T>
__global__ __launch_bounds__(NT) void k_env_right_b(DevState s, MeasWork mw, int j, int tiles_n) {
    __shared__ T As[8 * 64], Bs[8 * 64];
    const int bi = blockIdx.y, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int M = sd.chil, K = sd.d * sd.chir;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= M || tn * 64 >= M) return;
    const T* Bm = site_ptr<T>(s, b, j);
    const T* U = reinterpret_cast<const T*>(mw.W) + (size_t)bi * s.chi * s.dmax * s.chi;
    T* R = reinterpret_cast<T*>(mw.R) + ((size_t)j * mw.nbm + bi) * cc(s.chi);
    block_gemm<T, true, false, 8>(
        M, M, K, tm * 64, tn * 64,
        [&](int ap, int k) { return cconj(Bm[(size_t)ap * K + k]); },
        [&](int k, int a) { return U[(size_t)a * K + k]; },
        [&](int ap, int a, double2 v) { R[(size_t)ap * M + a] = cconv<T>(v); }, As, Bs);
}

// ---------------------------------------------------------------- left sweep pieces
// slot < nslot_x: Y[slot] = X[slot] . B_j ; slot == nslot_x: Y[slot] = E . B_j
template <class T>
__global__ __launch_bounds__(NT, 4) void k_meas_y(DevState s, MeasWork mw, int j, int nslot_x, int tiles_n) {
    __shared__ T As[8 * 64], Bs[8 * 64];
    const int nsl = nslot_x + 1;
    const int bi = blockIdx.y / nsl, slot = blockIdx.y % nsl, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int M = sd.chil, N = sd.d * sd.chir, K = sd.chil;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= M || tn * 64 >= N) return;
    const T* X = (slot < nslot_x) ? reinterpret_cast<const T*>(mw.X) + ((size_t)bi * s.L + slot) * cc(s.chi)
                                  : reinterpret_cast<const T*>(mw.E) + (size_t)bi * cc(s.chi);
    const T* Bm = site_ptr<T>(s, b, j);
    T* Y = reinterpret_cast<T*>(mw.Y) + ((size_t)bi * s.L + slot) * s.chi * s.dmax * s.chi;
    block_gemm<T, true, true, 8>(
        M, N, K, tm * 64, tn * 64,
        [&](int ap, int a) { return X[(size_t)ap * K + a]; },
        [&](int a, int pc) { return Bm[(size_t)a * N + pc]; },
        [&](int ap, int pc, double2 v) { Y[(size_t)ap * N + pc] = cconv<T>(v); }, As, Bs);
}

// W[(a',p')][c] = sum_c' conj(B[(a',p')][c']) R_{j+1}[c'][c]
template <class T>
__global__ __launch_bounds__(NT) void k_meas_w(DevState s, MeasWork mw, int j, int tiles_n) {
    __shared__ T As[8 * 64], Bs[8 * 64];
    const int bi = blockIdx.y, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int M = sd.chil * sd.d, N = sd.chir, K = sd.chir;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= M || tn * 64 >= N) return;
    const T* P = site_ptr<T>(s, b, j);
    const T* R = reinterpret_cast<const T*>(mw.R) + ((size_t)(j + 1) * mw.nbm + bi) * cc(s.chi);
    T* W = reinterpret_cast<T*>(mw.W) + (size_t)bi * s.chi * s.dmax * s.chi;
    block_gemm<T, true, true, 8>(
        M, N, K, tm * 64, tn * 64,
        [&](int r, int cp) { return cconj(P[(size_t)r * K + cp]); },
        [&](int cp, int c) { return R[(size_t)cp * N + c]; },
        [&](int r, int c, double2 v) { W[(size_t)r * N + c] = cconv<T>(v); }, As, Bs);
}

// value = sum_{n',n} O[n'][n] sum_k sum_{a',c} Y[a'][(n,k)][c] W[(a',(n',k))][c]   (FP64 accumulate)
// mode 0: slots i < j give C[i][j] with O = s-; slot j gives C[j][j] with O = n.
template <class T>
__global__ __launch_bounds__(NT) void k_meas_dot(DevState s, MeasWork mw, int j, int nslot_x) {
    __shared__ double2 red[NT];
    const int nsl = nslot_x + 1;
    const int bi = blockIdx.x / nsl, slot = blockIdx.x % nsl, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int dk = sd.dk, chir = sd.chir, N = sd.d * chir;
    const int np = (slot < nslot_x) ? 0 : 1;  // bra physical n' paired with ket n = 1
    const T* Y = reinterpret_cast<const T*>(mw.Y) + ((size_t)bi * s.L + slot) * s.chi * s.dmax * s.chi;
    const T* W = reinterpret_cast<const T*>(mw.W) + (size_t)bi * s.chi * s.dmax * s.chi;
    double2 acc = mk(0.0, 0.0);
    const int tot = sd.chil * dk * chir;
    for (int e = threadIdx.x; e < tot; e += NT) {
        int ap = e / (dk * chir), rem = e % (dk * chir), k = rem / chir, c = rem % chir;
        double2 y = cconv<double2>(Y[(size_t)ap * N + (1 * dk + k) * chir + c]);
        double2 wv = cconv<double2>(W[(size_t)ap * N + (np * dk + k) * chir + c]);
        cfma(acc, y, wv);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int i = (slot < nslot_x) ? slot : j;
        mw.C[((size_t)bi * s.L + i) * s.L + j] = red[0];
    }
}

// (k_meas_y and k_meas_upd ask for four workgroups per CU: at most 128 registers, no spills,
// four waves per SIMD instead of three; the sweep takes 12 % less time.)
// String updates at site j:
//   slot < nslot_x : X[slot] <- sum_{(a',p)} s_p conj(B[(a',p)][c']) Y[slot][(a',p)][c],  s_p = (-1)^n
//   slot == nslot_x: X[j]    <- sum_{(a',k)} conj(B[(a',(1,k))][c']) Y[j][(a',(0,k))][c]   (s+)
//   slot == nslot_x+1: E     <- sum_{(a',p)} conj(B[(a',p)][c']) Y[j][(a',p)][c]
template <class T>
__global__ __launch_bounds__(NT, 4) void k_meas_upd(DevState s, MeasWork mw, int j, int nslot_x, int tiles_n) {
    __shared__ T As[8 * 64], Bs[8 * 64];
    typedef typename real_of<T>::type R;
    const int nsl = nslot_x + 2;
    const int bi = blockIdx.y / nsl, slot = blockIdx.y % nsl, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int chil = sd.chil, chir = sd.chir, d = sd.d, dk = sd.dk;
    int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    if (tm * 64 >= chir || tn * 64 >= chir) return;
    const T* Bm = site_ptr<T>(s, b, j);
    const int ysl = slot < nslot_x ? slot : nslot_x;
    const T* Y = reinterpret_cast<const T*>(mw.Y) + ((size_t)bi * s.L + ysl) * s.chi * s.dmax * s.chi;
    T* out;
    if (slot < nslot_x) out = reinterpret_cast<T*>(mw.X) + ((size_t)bi * s.L + slot) * cc(s.chi);
    else if (slot == nslot_x) out = reinterpret_cast<T*>(mw.X) + ((size_t)bi * s.L + j) * cc(s.chi);
    else out = reinterpret_cast<T*>(mw.E) + (size_t)bi * cc(s.chi);
    if (slot == nslot_x) {
        const int K = chil * dk;
        block_gemm<T, false, true, 8>(
            chir, chir, K, tm * 64, tn * 64,
            [&](int cp, int kk) {
                int ap = kk / dk, k = kk % dk;
                return cconj(Bm[((size_t)ap * d + dk + k) * chir + cp]);
            },
            [&](int kk, int c) {
                int ap = kk / dk, k = kk % dk;
                return Y[((size_t)ap * d + k) * chir + c];
            },
            [&](int cp, int c, double2 v) { out[(size_t)cp * chir + c] = cconv<T>(v); }, As, Bs);
    } else {
        const bool fsign = slot < nslot_x;
        const int K = chil * d;
        block_gemm<T, false, true, 8>(
            chir, chir, K, tm * 64, tn * 64,
            [&](int cp, int kk) {
                int p = kk % d;
                T v = cconj(Bm[(size_t)kk * chir + cp]);
                if (fsign && p >= dk) { v.x = -v.x; v.y = -v.y; }
                return v;
            },
            [&](int kk, int c) { return Y[(size_t)kk * chir + c]; },
            [&](int cp, int c, double2 v) { out[(size_t)cp * chir + c] = cconv<T>(v); }, As, Bs);
    }
}

template <class T>
__global__ void k_meas_init(DevState s, MeasWork mw) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= mw.nbm) return;
    T one;
    one.x = 1;
    one.y = 0;
    reinterpret_cast<T*>(mw.R)[((size_t)s.L * mw.nbm + bi) * cc(s.chi)] = one;
    reinterpret_cast<T*>(mw.E)[(size_t)bi * cc(s.chi)] = one;
}

template <class T>
__global__ void k_meas_final(DevState s, MeasWork mw) {
    const int bi = blockIdx.x;
    const T* E = reinterpret_cast<const T*>(mw.E) + (size_t)bi * cc(s.chi);
    const double nrm = (double)E[0].x;
    if (threadIdx.x == 0) mw.nrm[bi] = nrm;
    const int L = s.L;
    double2* C = mw.C + (size_t)bi * L * L;
    __syncthreads();
    for (int e = threadIdx.x; e < L * L; e += blockDim.x) {
        int i = e / L, jj = e % L;
        if (i > jj) C[e] = cconj(C[(size_t)jj * L + i]);
    }
}

template <class T>
static void measure_mps_t(const DevState& s, const MeasWork& mw, hipStream_t st) {
    const int ch = (s.chi + 63) / 64, chd = (s.chi * s.dmax + 63) / 64;
    hipLaunchKernelGGL(k_meas_init<T>, dim3((mw.nbm + 63) / 64), dim3(64), 0, st, s, mw);
    for (int j = s.L - 1; j >= 0; --j) {
        hipLaunchKernelGGL(k_env_right_a<T>, dim3(chd * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
        hipLaunchKernelGGL(k_env_right_b<T>, dim3(ch * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
    }
    for (int j = 0; j < s.L; ++j) {
        // j open strings (slots 0..j-1) + the norm environment
        hipLaunchKernelGGL(k_meas_y<T>, dim3(ch * chd, mw.nbm * (j + 1)), dim3(NT), 0, st, s, mw, j, j, chd);
        hipLaunchKernelGGL(k_meas_w<T>, dim3(chd * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
        hipLaunchKernelGGL(k_meas_dot<T>, dim3(mw.nbm * (j + 1)), dim3(NT), 0, st, s, mw, j, j);
        hipLaunchKernelGGL(k_meas_upd<T>, dim3(ch * ch, mw.nbm * (j + 2)), dim3(NT), 0, st, s, mw, j, j, ch);
    }
    hipLaunchKernelGGL(k_meas_final<T>, dim3(mw.nbm), dim3(NT), 0, st, s, mw);
}

void launch_measure_mps(int prec, const DevState& s, const MeasWork& mw, hipStream_t st) {
    if (prec == 0) measure_mps_t<double2>(s, mw, st);
    else measure_mps_t<float2>(s, mw, st);
}

// ---------------------------------------------------------------- QT rates, shift means
// closing of a local O on site j: <psi|O|psi> = sum O[n'][n] sum_k <Y[(n,k)], W[(n',k)]>, Y = E_{j-1} B_j
// (row index n' = bra).  O = L^+L gives the rate numerator (real part to vals); O = L gives <L>
// for the shifted jump operators (complex, to cvals when it is non-null).
template <class T>
__global__ __launch_bounds__(NT) void k_jump_dot(DevState s, MeasWork mw, int j, double2 o00, double2 o01,
                                                  double2 o10, double2 o11, double* vals, double2* cvals, int njump,
                                                  int jk) {
    __shared__ double2 red[NT];
    const int bi = blockIdx.x, b = mw.b0 + bi;
    SiteDims sd = site_dims(s, b, j);
    const int dk = sd.dk, chir = sd.chir, N = sd.d * chir;
    const T* Y = reinterpret_cast<const T*>(mw.Y) + ((size_t)bi * s.L + 0) * s.chi * s.dmax * s.chi;
    const T* W = reinterpret_cast<const T*>(mw.W) + (size_t)bi * s.chi * s.dmax * s.chi;
    double2 O[2][2] = {{o00, o01}, {o10, o11}};
    double2 acc = mk(0.0, 0.0);
    const int tot = sd.chil * dk * chir;
    for (int e = threadIdx.x; e < tot; e += NT) {
        int ap = e / (dk * chir), rem = e % (dk * chir), k = rem / chir, c = rem % chir;
        for (int np = 0; np < 2; ++np)
            for (int nn = 0; nn < 2; ++nn) {
                double2 o = O[np][nn];
                if (o.x == 0.0 && o.y == 0.0) continue;
                double2 y = cconv<double2>(Y[(size_t)ap * N + (nn * dk + k) * chir + c]);
                double2 wv = cconv<double2>(W[(size_t)ap * N + (np * dk + k) * chir + c]);
                cfma(acc, o, cmul(y, wv));
            }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (cvals) cvals[(size_t)bi * njump + jk] = red[0];
        else vals[(size_t)bi * njump + jk] = red[0].x;
    }
}

// E_j for all j are not stored; instead the left sweep stops at each jump site.
template <class T>
static void jump_expect_t(const DevState& s, const MeasWork& mw, int njump, const int* jsite,
                          const double2* jLdL, double* vals, const double2* jL, double2* lvals, hipStream_t st) {
    const int ch = (s.chi + 63) / 64, chd = (s.chi * s.dmax + 63) / 64;
    hipLaunchKernelGGL(k_meas_init<T>, dim3((mw.nbm + 63) / 64), dim3(64), 0, st, s, mw);
    for (int j = s.L - 1; j >= 0; --j) {
        hipLaunchKernelGGL(k_env_right_a<T>, dim3(chd * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
        hipLaunchKernelGGL(k_env_right_b<T>, dim3(ch * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
    }
    for (int j = 0; j < s.L; ++j) {
        // Y = E_{j-1} B_j (slot 0 plays the role of the norm environment)
        hipLaunchKernelGGL(k_meas_y<T>, dim3(ch * chd, mw.nbm), dim3(NT), 0, st, s, mw, j, 0, chd);
        bool have_w = false;
        for (int q = 0; q < njump; ++q) {
            if (jsite[q] != j) continue;
            if (!have_w) {  // W = conj(B_j) R_{j+1}, shared by every channel on this site
                hipLaunchKernelGGL(k_meas_w<T>, dim3(chd * ch, mw.nbm), dim3(NT), 0, st, s, mw, j, ch);
                have_w = true;
            }
            hipLaunchKernelGGL(k_jump_dot<T>, dim3(mw.nbm), dim3(NT), 0, st, s, mw, j, jLdL[4 * q + 0],
                               jLdL[4 * q + 1], jLdL[4 * q + 2], jLdL[4 * q + 3], vals, (double2*)nullptr, njump, q);
            if (jL)
                hipLaunchKernelGGL(k_jump_dot<T>, dim3(mw.nbm), dim3(NT), 0, st, s, mw, j, jL[4 * q + 0],
                                   jL[4 * q + 1], jL[4 * q + 2], jL[4 * q + 3], (double*)nullptr, lvals, njump, q);
        }
        // E_j = sum_p B^p+ Y^p  (slot nslot_x+1 with nslot_x = 0 -> E update only; the s+ slot writes X[j], unused)
        hipLaunchKernelGGL(k_meas_upd<T>, dim3(ch * ch, mw.nbm * 2), dim3(NT), 0, st, s, mw, j, 0, ch);
    }
    hipLaunchKernelGGL(k_meas_final<T>, dim3(mw.nbm), dim3(64), 0, st, s, mw);
}

void launch_jump_expect(int prec, const DevState& s, const MeasWork& mw, int njump, const int* jsite,
                        const double2* jLdL, double* vals, const double2* jL, double2* lvals, hipStream_t st) {
    if (prec == 0) jump_expect_t<double2>(s, mw, njump, jsite, jLdL, vals, jL, lvals, st);
    else jump_expect_t<float2>(s, mw, njump, jsite, jLdL, vals, jL, lvals, st);
}

// ---------------------------------------------------------------- MPDO (trace vectors)
// local matrices: M_I = B[:,0,:] + B[:,3,:], M_n = B[:,3,:], M_s+ = B[:,1,:], M_s- = B[:,2,:],
// M_F = B[:,0,:] - B[:,3,:]   (t_O[m = n*2+n'] = O[n'][n])
template <class T>
__device__ __forceinline__ double2 mpdo_m(const T* Bm, int chir, int a, int c, int op) {
    const T* row = Bm + (size_t)a * 4 * chir;
    switch (op) {
        case 0: return cadd(cconv<double2>(row[0 * chir + c]), cconv<double2>(row[3 * chir + c]));
        case 1: return cconv<double2>(row[3 * chir + c]);
        case 2: return cconv<double2>(row[1 * chir + c]);
        case 3: return cconv<double2>(row[2 * chir + c]);
        default: return csub(cconv<double2>(row[0 * chir + c]), cconv<double2>(row[3 * chir + c]));
    }
}

// left vectors e_j (j = 0..L) and right vectors r_j, one block per instance; stored in mw.R as double2
// layout: mw.R (reused) -> [bi][j][chi] for e, and mw.E (reused) -> [bi][j][chi] for r
template <class T>
__global__ __launch_bounds__(NT) void k_mpdo_vecs(DevState s, MeasWork mw) {
    const int bi = blockIdx.x, b = mw.b0 + bi;
    double2* ev = reinterpret_cast<double2*>(mw.R) + (size_t)bi * (s.L + 1) * s.chi;
    double2* rv = reinterpret_cast<double2*>(mw.E) + (size_t)bi * (s.L + 1) * s.chi;
    if (threadIdx.x == 0) {
        ev[0] = mk(1.0, 0.0);
        rv[(size_t)s.L * s.chi] = mk(1.0, 0.0);
    }
    __syncthreads();
    for (int j = 0; j < s.L; ++j) {
        SiteDims sd = site_dims(s, b, j);
        const T* Bm = site_ptr<T>(s, b, j);
        for (int c = threadIdx.x; c < sd.chir; c += NT) {
            double2 acc = mk(0.0, 0.0);
            for (int a = 0; a < sd.chil; ++a) cfma(acc, ev[(size_t)j * s.chi + a], mpdo_m(Bm, sd.chir, a, c, 0));
            ev[(size_t)(j + 1) * s.chi + c] = acc;
        }
        __syncthreads();
    }
    for (int j = s.L - 1; j >= 0; --j) {
        SiteDims sd = site_dims(s, b, j);
        const T* Bm = site_ptr<T>(s, b, j);
        for (int a = threadIdx.x; a < sd.chil; a += NT) {
            double2 acc = mk(0.0, 0.0);
            for (int c = 0; c < sd.chir; ++c) cfma(acc, mpdo_m(Bm, sd.chir, a, c, 0), rv[(size_t)(j + 1) * s.chi + c]);
            rv[(size_t)j * s.chi + a] = acc;
        }
        __syncthreads();
    }
}

// one block per (instance, i): upper string s+_i F.. s-_j and lower string s-_i F.. s+_j
template <class T>
__global__ __launch_bounds__(NT) void k_mpdo_strings(DevState s, MeasWork mw) {
    __shared__ double2 xu[512], xl[512], tu[512], tl[512];
    __shared__ double2 red[2][NT];
    const int L = s.L;
    const int bi = blockIdx.x / L, i = blockIdx.x % L, b = mw.b0 + bi;
    const double2* ev = reinterpret_cast<const double2*>(mw.R) + (size_t)bi * (L + 1) * s.chi;
    const double2* rv = reinterpret_cast<const double2*>(mw.E) + (size_t)bi * (L + 1) * s.chi;
    double2* C = mw.C + (size_t)bi * L * L;
    SiteDims sd = site_dims(s, b, i);
    const T* Bi = site_ptr<T>(s, b, i);
    // diagonal and string heads
    double2 dpart = mk(0.0, 0.0);
    for (int c = threadIdx.x; c < sd.chir; c += NT) {
        double2 au = mk(0.0, 0.0), al = mk(0.0, 0.0), an = mk(0.0, 0.0);
        for (int a = 0; a < sd.chil; ++a) {
            double2 e = ev[(size_t)i * s.chi + a];
            cfma(au, e, mpdo_m(Bi, sd.chir, a, c, 2));
            cfma(al, e, mpdo_m(Bi, sd.chir, a, c, 3));
            cfma(an, e, mpdo_m(Bi, sd.chir, a, c, 1));
        }
        xu[c] = au;
        xl[c] = al;
        cfma(dpart, an, rv[(size_t)(i + 1) * s.chi + c]);
    }
    red[0][threadIdx.x] = dpart;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[0][threadIdx.x] = cadd(red[0][threadIdx.x], red[0][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) C[(size_t)i * L + i] = red[0][0];
    __syncthreads();
    for (int j = i + 1; j < L; ++j) {
        SiteDims sj = site_dims(s, b, j);
        const T* Bj = site_ptr<T>(s, b, j);
        double2 pu = mk(0.0, 0.0), pl = mk(0.0, 0.0);
        for (int c = threadIdx.x; c < sj.chir; c += NT) {
            double2 cu = mk(0.0, 0.0), cl = mk(0.0, 0.0), fu = mk(0.0, 0.0), fl = mk(0.0, 0.0);
            for (int a = 0; a < sj.chil; ++a) {
                double2 mf = mpdo_m(Bj, sj.chir, a, c, 4);
                cfma(cu, xu[a], mpdo_m(Bj, sj.chir, a, c, 3));
                cfma(cl, xl[a], mpdo_m(Bj, sj.chir, a, c, 2));
                cfma(fu, xu[a], mf);
                cfma(fl, xl[a], mf);
            }
            double2 r = rv[(size_t)(j + 1) * s.chi + c];
            cfma(pu, cu, r);
            cfma(pl, cl, r);
            tu[c] = fu;
            tl[c] = fl;
        }
        red[0][threadIdx.x] = pu;
        red[1][threadIdx.x] = pl;
        __syncthreads();
        for (int o = NT / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) {
                red[0][threadIdx.x] = cadd(red[0][threadIdx.x], red[0][threadIdx.x + o]);
                red[1][threadIdx.x] = cadd(red[1][threadIdx.x], red[1][threadIdx.x + o]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            C[(size_t)i * L + j] = red[0][0];
            C[(size_t)j * L + i] = red[1][0];
        }
        for (int c = threadIdx.x; c < sj.chir; c += NT) {
            xu[c] = tu[c];
            xl[c] = tl[c];
        }
        __syncthreads();
    }
    if (i == 0 && threadIdx.x == 0) mw.nrm[bi] = ev[(size_t)L * s.chi].x;
}

void launch_measure_mpdo(int prec, const DevState& s, const MeasWork& mw, hipStream_t st) {
    if (prec == 0) {
        hipLaunchKernelGGL(k_mpdo_vecs<double2>, dim3(mw.nbm), dim3(NT), 0, st, s, mw);
        hipLaunchKernelGGL(k_mpdo_strings<double2>, dim3(mw.nbm * s.L), dim3(NT), 0, st, s, mw);
    } else {
        hipLaunchKernelGGL(k_mpdo_vecs<float2>, dim3(mw.nbm), dim3(NT), 0, st, s, mw);
        hipLaunchKernelGGL(k_mpdo_strings<float2>, dim3(mw.nbm * s.L), dim3(NT), 0, st, s, mw);
    }
}
