// Dissipative part of a time step (gfx950).
//   quantum trajectories  (Sec. 4.1): jump choice from FP64 rates and uniforms, L_k applied locally;
//   quantum state diffusion (Sec. 4.2): local factors 1 + dW_k sqrt(gamma_k) L_k, linear unravelling;
//   both optionally with the shifted operators L_k - <L_k> and their drift (Sec. 4.1, 4.2);
//   Kraus compression of the locally purified form (Sec. 3.2): new Kraus columns from the
//   2chi_k x 2chi_k Gram matrix of M = [A | sqrt(gamma dt) L A], weighted by the left bond
//   weights of the site (its environment in the Hastings form).
#include "common.h"
#include "launch.h"
#include <float.h>

// B[a][(n,k)][c] <- sum_m O[n][m] B[a][(m,k)][c]   for one instance (block) and one site
template <class T>
__device__ void apply_local(const DevState& s, int b, int site, double2 o00, double2 o01, double2 o10, double2 o11) {
    T* Bm = site_ptr<T>(s, b, site);
    const int chil = bond_dim(s, b, site), chir = bond_dim(s, b, site + 1);
    const int d = s.dsite[site], dk = d / 2;
    const int tot = chil * dk * chir;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        int a = e / (dk * chir), rem = e % (dk * chir), k = rem / chir, c = rem % chir;
        size_t i0 = ((size_t)a * d + 0 * dk + k) * chir + c;
        size_t i1 = ((size_t)a * d + 1 * dk + k) * chir + c;
        double2 x0 = cconv<double2>(Bm[i0]), x1 = cconv<double2>(Bm[i1]);
        double2 y0 = mk(0, 0), y1 = mk(0, 0);
        cfma(y0, o00, x0); cfma(y0, o01, x1);
        cfma(y1, o10, x0); cfma(y1, o11, x1);
        Bm[i0] = cconv<T>(y0);
        Bm[i1] = cconv<T>(y1);
    }
}

// one block per instance of the chunk: decide and apply the jump.
// Shifted operators (Sec. 4.1, lvals != null, l_k = lvals/nrm the normalized <L_k>): rates
// gamma_k dt (<L_k^+L_k> - |l_k|^2), a jump applies L_k - l_k, and without a jump every channel's
// factor 1 + dt gamma_k (conj(l_k) L_k - |l_k|^2/2) (the state-dependent single-site part of the
// shifted h^eff, first order) is applied in channel order before the h^eff Trotter step.
template <class T>
__global__ void k_qt_apply(DevState s, int b0, double dt, int njump, const int* jsite, const double2* jop,
                           const double* gam, const double* vals, const double2* lvals, const double* nrm,
                           const double* rnd, int* jumped, unsigned char* mask) {
    const int bi = blockIdx.x, b = b0 + bi;
    __shared__ int sk;
    const double nr = nrm[bi];
    if (threadIdx.x == 0) {
        const double u = rnd[b];
        double cum = 0.0;
        int k = -1;
        for (int q = 0; q < njump; ++q) {
            double m = vals[(size_t)bi * njump + q] / nr;
            if (lvals) {
                const double2 l = cscale(lvals[(size_t)bi * njump + q], 1.0 / nr);
                m -= l.x * l.x + l.y * l.y;
            }
            cum += gam[q] * dt * m;
            if (u < cum) { k = q; break; }
        }
        sk = k;
        jumped[b] = k;
        mask[b] = (k >= 0) ? 1 : 0;
        // normalized state afterwards: jumped -> norm^2 = <L^+L> (shifted: nrm (m - |l|^2)), else <B|B>
        double n2 = nr;
        if (k >= 0) {
            n2 = vals[(size_t)bi * njump + k];
            if (lvals) {
                const double2 l = cscale(lvals[(size_t)bi * njump + k], 1.0 / nr);
                n2 = nr * (n2 / nr - (l.x * l.x + l.y * l.y));
            }
        }
        s.lognorm[b] = -0.5 * log(n2);
    }
    __syncthreads();
    const int k = sk;
    if (k >= 0) {
        const double2* o = jop + 4 * k;
        double2 l = mk(0.0, 0.0);
        if (lvals) l = cscale(lvals[(size_t)bi * njump + k], 1.0 / nr);
        apply_local<T>(s, b, jsite[k], csub(o[0], l), o[1], o[2], csub(o[3], l));
    } else if (lvals) {
        for (int q = 0; q < njump; ++q) {
            const double2* o = jop + 4 * q;
            const double2 l = cscale(lvals[(size_t)bi * njump + q], 1.0 / nr);
            const double c = dt * gam[q], h = 0.5 * c * (l.x * l.x + l.y * l.y);
            const double2 cl = cscale(cconj(l), c);
            apply_local<T>(s, b, jsite[q], cadd(mk(1.0 - h, 0.0), cmul(cl, o[0])), cmul(cl, o[1]), cmul(cl, o[2]),
                           cadd(mk(1.0 - h, 0.0), cmul(cl, o[3])));
            __syncthreads();
        }
    }
}

void launch_qt_apply(int prec, const DevState& s, int b0, int nbm, double dt, int njump, const int* jsite,
                     const double2* jop, const double* gam, const double* vals, const double2* lvals,
                     const double* nrm, const double* rnd, int* jumped, unsigned char* mask, hipStream_t st) {
    if (prec == 0)
        hipLaunchKernelGGL(k_qt_apply<double2>, dim3(nbm), dim3(256), 0, st, s, b0, dt, njump, jsite, jop, gam, vals,
                           lvals, nrm, rnd, jumped, mask);
    else
        hipLaunchKernelGGL(k_qt_apply<float2>, dim3(nbm), dim3(256), 0, st, s, b0, dt, njump, jsite, jop, gam, vals,
                           lvals, nrm, rnd, jumped, mask);
}

// one block per (instance, jump): psi <- (1 + dW sqrt(gamma) L) psi on the jump site.
// Shifted (Sec. 4.2, lvals != null): psi <- (1 + dW sqrt(gamma)(L - l)) (1 + dt gamma (conj(l) L - |l|^2/2)) psi
// with l = lvals/nrm, the normalized <L> of the state before the step's first factor.
template <class T>
__global__ void k_qsd_apply(DevState s, int b0, double dt, int njump, int q, const int* jsite, const double2* jop,
                            const double* gam, const double* rnd, int noise_kind, const double2* lvals,
                            const double* nrm) {
    const int bi = blockIdx.x, b = b0 + bi;
    double2 dW;
    if (noise_kind == 0) {
        double x = rnd[((size_t)b * njump + q) * 2 + 0], y = rnd[((size_t)b * njump + q) * 2 + 1];
        double sc = sqrt(dt) / sqrt(2.0);
        dW = mk(x * sc, y * sc);
    } else {
        double u = rnd[(size_t)b * njump + q];
        dW = mk(u < 0.5 ? -sqrt(dt) : sqrt(dt), 0.0);
    }
    const double sg = sqrt(gam[q]);
    const double2* o = jop + 4 * q;
    double2 f = cscale(dW, sg);
    double2 m00 = cadd(mk(1, 0), cmul(f, o[0]));
    double2 m01 = cmul(f, o[1]);
    double2 m10 = cmul(f, o[2]);
    double2 m11 = cadd(mk(1, 0), cmul(f, o[3]));
    if (lvals) {
        const double2 l = cscale(lvals[(size_t)bi * njump + q], 1.0 / nrm[bi]);
        const double2 fl = cmul(f, l);
        m00 = csub(m00, fl);
        m11 = csub(m11, fl);
        const double c = dt * gam[q], h = 0.5 * c * (l.x * l.x + l.y * l.y);
        const double2 cl = cscale(cconj(l), c);
        const double2 d00 = cadd(mk(1.0 - h, 0.0), cmul(cl, o[0])), d01 = cmul(cl, o[1]);
        const double2 d10 = cmul(cl, o[2]), d11 = cadd(mk(1.0 - h, 0.0), cmul(cl, o[3]));
        const double2 n00 = cadd(cmul(m00, d00), cmul(m01, d10)), n01 = cadd(cmul(m00, d01), cmul(m01, d11));
        const double2 n10 = cadd(cmul(m10, d00), cmul(m11, d10)), n11 = cadd(cmul(m10, d01), cmul(m11, d11));
        m00 = n00; m01 = n01; m10 = n10; m11 = n11;
    }
    apply_local<T>(s, b, jsite[q], m00, m01, m10, m11);
}

void launch_qsd_apply(int prec, const DevState& s, int b0, int nbm, double dt, int njump, const int* jsite,
                      const double2* jop, const double* gam, const double* rnd, int noise_kind, const double2* lvals,
                      const double* nrm, hipStream_t st) {
    // one launch per jump: factors acting on the same site are applied in jump order
    for (int q = 0; q < njump; ++q) {
        if (prec == 0)
            hipLaunchKernelGGL(k_qsd_apply<double2>, dim3(nbm), dim3(256), 0, st, s, b0, dt, njump, q, jsite, jop,
                               gam, rnd, noise_kind, lvals, nrm);
        else
            hipLaunchKernelGGL(k_qsd_apply<float2>, dim3(nbm), dim3(256), 0, st, s, b0, dt, njump, q, jsite, jop,
                               gam, rnd, noise_kind, lvals, nrm);
    }
}

// ---------------------------------------------------------------- Kraus compression
// Site tensor A[a][(n,k)][c], dk Kraus columns (dk = d/2 = chi_k).  M = [A | sqrt(gamma dt) L A]
// has rows (a, n, c) and 2dk columns.  G = Mw^+ Mw with Mw = Lambda_{site-1}[a] M;
// cyclic Jacobi on G (FP64), keep the dk eigenvectors of largest eigenvalue: A_new = M W.
#define KMAX 16
template <class T>
__global__ __launch_bounds__(256) void k_kraus(DevState s, double dt, int q, int site, double2 l00, double2 l01,
                                                double2 l10, double2 l11, double gamma) {
    __shared__ double2 G[KMAX][KMAX];
    __shared__ double2 Wv[KMAX][KMAX];
    __shared__ double2 red[256];
    __shared__ int order[KMAX];
    const int b = blockIdx.x;
    T* Bm = site_ptr<T>(s, b, site);
    const int chil = bond_dim(s, b, site), chir = bond_dim(s, b, site + 1);
    const int d = s.dsite[site], dk = d / 2, kk = 2 * dk;
    const double* lamL = site > 0 ? lam_ptr(s, b, site - 1) : nullptr;
    const double sq = sqrt(gamma * dt);
    const int rows = chil * 2 * chir;
    // M(row, col): row = (a, n, c); col < dk: A[a][(n,col)][c]; col >= dk: sqrt(g dt) (L A)[a][(n,col-dk)][c]
    auto Mval = [&](int row, int col) -> double2 {
        int a = row / (2 * chir), rem = row % (2 * chir), n = rem / chir, c = rem % chir;
        int k = col < dk ? col : col - dk;
        double2 x0 = cconv<double2>(Bm[((size_t)a * d + 0 * dk + k) * chir + c]);
        double2 x1 = cconv<double2>(Bm[((size_t)a * d + 1 * dk + k) * chir + c]);
        if (col < dk) return n == 0 ? x0 : x1;
        double2 y = mk(0, 0);
        if (n == 0) { cfma(y, l00, x0); cfma(y, l01, x1); }
        else { cfma(y, l10, x0); cfma(y, l11, x1); }
        return cscale(y, sq);
    };
    for (int p = 0; p < kk; ++p)
        for (int qq = p; qq < kk; ++qq) {
            double2 acc = mk(0, 0);
            for (int r = threadIdx.x; r < rows; r += 256) {
                double wl = 1.0;
                if (lamL) { double l = lamL[r / (2 * chir)]; wl = l * l; }
                cfmac(acc, Mval(r, p), cscale(Mval(r, qq), wl));
            }
            red[threadIdx.x] = acc;
            __syncthreads();
            for (int o = 128; o > 0; o >>= 1) {
                if (threadIdx.x < o) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + o]);
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                G[p][qq] = red[0];
                G[qq][p] = cconj(red[0]);
            }
            __syncthreads();
        }
    if (threadIdx.x == 0) {
        for (int p = 0; p < kk; ++p)
            for (int qq = 0; qq < kk; ++qq) Wv[p][qq] = mk(p == qq ? 1.0 : 0.0, 0.0);
        for (int p = 0; p < kk; ++p) G[p][p].y = 0.0;
        // cyclic complex Jacobi: for each pair, phase D = diag(1, e^{-i phi}) makes the pair block real,
        // then a real rotation diagonalizes it (R = D P)
        for (int sweep = 0; sweep < 50; ++sweep) {
            double off = 0.0, dia = 0.0;
            for (int p = 0; p < kk; ++p) {
                dia += G[p][p].x * G[p][p].x;
                for (int qq = p + 1; qq < kk; ++qq) off += G[p][qq].x * G[p][qq].x + G[p][qq].y * G[p][qq].y;
            }
            if (off <= 1e-32 * dia || off == 0.0) break;
            for (int p = 0; p < kk; ++p)
                for (int qq = p + 1; qq < kk; ++qq) {
                    double2 g = G[p][qq];
                    double ag = sqrt(g.x * g.x + g.y * g.y);
                    if (ag == 0.0) continue;
                    double2 ph = mk(g.x / ag, g.y / ag);  // e^{i phi}
                    double app = G[p][p].x, aqq = G[qq][qq].x;
                    double zeta = (aqq - app) / (2.0 * ag);
                    double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                    // R columns: r_p = (cs) e_p + (-sn e^{-i phi}) e_q ; r_q = (sn) e_p + (cs e^{-i phi}) e_q
                    double2 em = cconj(ph);
                    double2 rpp = mk(cs, 0), rqp = cscale(em, -sn), rpq = mk(sn, 0), rqq = cscale(em, cs);
                    // G <- G R (columns p, q)
                    for (int r = 0; r < kk; ++r) {
                        double2 gp = G[r][p], gq = G[r][qq];
                        double2 np_ = cadd(cmul(gp, rpp), cmul(gq, rqp));
                        double2 nq_ = cadd(cmul(gp, rpq), cmul(gq, rqq));
                        G[r][p] = np_;
                        G[r][qq] = nq_;
                        double2 vp = Wv[r][p], vq = Wv[r][qq];
                        Wv[r][p] = cadd(cmul(vp, rpp), cmul(vq, rqp));
                        Wv[r][qq] = cadd(cmul(vp, rpq), cmul(vq, rqq));
                    }
                    // G <- R^+ G (rows p, q)
                    for (int c = 0; c < kk; ++c) {
                        double2 gp = G[p][c], gq = G[qq][c];
                        double2 np_ = cadd(cmulc(rpp, gp), cmulc(rqp, gq));
                        double2 nq_ = cadd(cmulc(rpq, gp), cmulc(rqq, gq));
                        G[p][c] = np_;
                        G[qq][c] = nq_;
                    }
                    G[p][qq] = mk(0, 0);
                    G[qq][p] = mk(0, 0);
                }
        }
        // order eigenvalues descending (stable)
        for (int p = 0; p < kk; ++p) {
            int rk = 0;
            for (int qq = 0; qq < kk; ++qq)
                rk += (G[qq][qq].x > G[p][p].x || (G[qq][qq].x == G[p][p].x && qq < p)) ? 1 : 0;
            if (rk < dk) order[rk] = p;
        }
    }
    __syncthreads();
    // A_new[a][(n,k)][c] = sum_col M((a,n,c), col) W[col][order[k]]; each thread owns one (a, c) pair
    // and both of its rows n = 0, 1, so the tensor is read completely before it is overwritten
    const int npair = chil * chir;
    for (int e = threadIdx.x; e < npair; e += 256) {
        const int a = e / chir, c = e % chir;
        double2 x0[KMAX / 2], x1[KMAX / 2];
        for (int k = 0; k < dk; ++k) {
            x0[k] = cconv<double2>(Bm[((size_t)a * d + 0 * dk + k) * chir + c]);
            x1[k] = cconv<double2>(Bm[((size_t)a * d + 1 * dk + k) * chir + c]);
        }
        for (int n = 0; n < 2; ++n) {
            double2 mrow[KMAX];
            for (int k = 0; k < dk; ++k) {
                mrow[k] = n == 0 ? x0[k] : x1[k];
                double2 y = mk(0, 0);
                if (n == 0) { cfma(y, l00, x0[k]); cfma(y, l01, x1[k]); }
                else { cfma(y, l10, x0[k]); cfma(y, l11, x1[k]); }
                mrow[dk + k] = cscale(y, sq);
            }
            for (int k = 0; k < dk; ++k) {
                double2 acc = mk(0, 0);
                for (int col = 0; col < kk; ++col) cfma(acc, mrow[col], Wv[col][order[k]]);
                Bm[((size_t)a * d + n * dk + k) * chir + c] = cconv<T>(acc);
            }
        }
    }
}

void launch_kraus(int prec, const DevState& s, double dt, int njump, const int* jsite, const double2* jop,
                  const double* gam, int chik, hipStream_t st) {
    for (int q = 0; q < njump; ++q) {
        const double2* o = jop + 4 * q;
        if (prec == 0)
            hipLaunchKernelGGL(k_kraus<double2>, dim3(s.B), dim3(256), 0, st, s, dt, q, jsite[q], o[0], o[1], o[2],
                               o[3], gam[q]);
        else
            hipLaunchKernelGGL(k_kraus<float2>, dim3(s.B), dim3(256), 0, st, s, dt, q, jsite[q], o[0], o[1], o[2],
                               o[3], gam[q]);
    }
}
