// Host-side FP64 construction of the Trotter bond gates.
//
//   exp(-i h^eff_b tau)  pure states, trajectories, diffusion and the purified form
//                        (Sec. 2.3; h^eff from eq. EffHamiltonian with each jump's
//                        -i/2 gamma L^+L shared between the bonds touching its site as in
//                        eq. LindbladLocal: a full share at a chain end, half in the bulk);
//   exp(l_b tau)         vectorized density matrix (Sec. 3.1 eq. Liouvillian with the
//                        row-major map A rho B -> A (x) B^T, so L rho L^+ -> L (x) L^*),
//                        returned in the basis of the local indices m = n*2 + n'.
// The matrix exponential is the scaling-and-squaring [13/13] Pade method of
// N. J. Higham, SIAM J. Matrix Anal. Appl. 26 (2005) 1179.
#include "host_gates.h"

#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

typedef std::complex<double> cd;

namespace {

struct Mat {
    int n;
    std::vector<cd> a;
    explicit Mat(int n_ = 0) : n(n_), a((size_t)n_ * n_, cd(0, 0)) {}
    cd& operator()(int i, int j) { return a[(size_t)i * n + j]; }
    cd operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

Mat eye(int n) {
    Mat m(n);
    for (int i = 0; i < n; ++i) m(i, i) = 1.0;
    return m;
}
Mat mul(const Mat& x, const Mat& y) {
    Mat r(x.n);
    for (int i = 0; i < x.n; ++i)
        for (int k = 0; k < x.n; ++k) {
            cd v = x(i, k);
            if (v == cd(0, 0)) continue;
            for (int j = 0; j < x.n; ++j) r(i, j) += v * y(k, j);
        }
    return r;
}
Mat add(const Mat& x, const Mat& y, cd sy = 1.0) {
    Mat r(x.n);
    for (size_t i = 0; i < x.a.size(); ++i) r.a[i] = x.a[i] + sy * y.a[i];
    return r;
}
Mat scal(const Mat& x, cd s) {
    Mat r(x.n);
    for (size_t i = 0; i < x.a.size(); ++i) r.a[i] = s * x.a[i];
    return r;
}
double norm1(const Mat& x) {
    double best = 0;
    for (int j = 0; j < x.n; ++j) {
        double s = 0;
        for (int i = 0; i < x.n; ++i) s += std::abs(x(i, j));
        best = std::max(best, s);
    }
    return best;
}
// solve P X = Q (Gaussian elimination with partial pivoting)
Mat solve(Mat P, Mat Q) {
    const int n = P.n;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(P(r, c)) > std::abs(P(piv, c))) piv = r;
        if (std::abs(P(piv, c)) == 0.0) throw std::runtime_error("singular Pade denominator");
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(P(c, j), P(piv, j));
                std::swap(Q(c, j), Q(piv, j));
            }
        for (int r = c + 1; r < n; ++r) {
            cd f = P(r, c) / P(c, c);
            if (f == cd(0, 0)) continue;
            for (int j = c; j < n; ++j) P(r, j) -= f * P(c, j);
            for (int j = 0; j < n; ++j) Q(r, j) -= f * Q(c, j);
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int j = 0; j < n; ++j) {
            cd v = Q(c, j);
            for (int k = c + 1; k < n; ++k) v -= P(c, k) * Q(k, j);
            Q(c, j) = v / P(c, c);
        }
    }
    return Q;
}

Mat expm(const Mat& A) {
    static const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                                 1187353796428800.0,  129060195264000.0,   10559470521600.0,
                                 670442572800.0,      33522128640.0,       1323241920.0,
                                 40840800.0,          960960.0,            16380.0,
                                 182.0,               1.0};
    const double theta13 = 5.371920351148152;
    const int n = A.n;
    double nrm = norm1(A);
    int sq = 0;
    if (nrm > theta13) sq = (int)std::ceil(std::log2(nrm / theta13));
    Mat X = scal(A, std::pow(2.0, -sq));
    Mat I = eye(n);
    Mat X2 = mul(X, X), X4 = mul(X2, X2), X6 = mul(X4, X2);
    Mat U1 = add(add(scal(X6, b[13]), scal(X4, b[11])), scal(X2, b[9]));
    Mat U2 = add(add(add(scal(X6, b[7]), scal(X4, b[5])), scal(X2, b[3])), scal(I, b[1]));
    Mat U = mul(X, add(mul(X6, U1), U2));
    Mat V1 = add(add(scal(X6, b[12]), scal(X4, b[10])), scal(X2, b[8]));
    Mat V2 = add(add(add(scal(X6, b[6]), scal(X4, b[4])), scal(X2, b[2])), scal(I, b[0]));
    Mat V = add(mul(X6, V1), V2);
    Mat R = solve(add(V, U, -1.0), add(V, U));
    for (int i = 0; i < sq; ++i) R = mul(R, R);
    return R;
}

Mat kron(const Mat& x, const Mat& y) {
    Mat r(x.n * y.n);
    for (int i = 0; i < x.n; ++i)
        for (int j = 0; j < x.n; ++j)
            for (int k = 0; k < y.n; ++k)
                for (int l = 0; l < y.n; ++l) r(i * y.n + k, j * y.n + l) = x(i, j) * y(k, l);
    return r;
}
Mat dagger(const Mat& x) {
    Mat r(x.n);
    for (int i = 0; i < x.n; ++i)
        for (int j = 0; j < x.n; ++j) r(i, j) = std::conj(x(j, i));
    return r;
}
Mat transpose(const Mat& x) {
    Mat r(x.n);
    for (int i = 0; i < x.n; ++i)
        for (int j = 0; j < x.n; ++j) r(i, j) = x(j, i);
    return r;
}
Mat conjm(const Mat& x) {
    Mat r(x.n);
    for (size_t i = 0; i < x.a.size(); ++i) r.a[i] = std::conj(x.a[i]);
    return r;
}

Mat from_interleaved(const double* p, int n) {
    Mat m(n);
    for (int i = 0; i < n * n; ++i) m.a[i] = cd(p[2 * i], p[2 * i + 1]);
    return m;
}

// weight of the on-site term of `site` given to bond b (eq. LindbladLocal)
double bond_share(int L, int site, int b) {
    int cnt = 0;
    bool has = false;
    for (int bb = site - 1; bb <= site; ++bb)
        if (bb >= 0 && bb <= L - 2) {
            ++cnt;
            if (bb == b) has = true;
        }
    return has ? 1.0 / cnt : 0.0;
}

Mat heff_bond(const TnModelHost& m, int b) {
    Mat h = from_interleaved(m.h_bond.data() + (size_t)b * 32, 4);
    Mat I2 = eye(2);
    for (size_t q = 0; q < m.jump_site.size(); ++q) {
        double w = bond_share(m.L, m.jump_site[q], b);
        if (w == 0.0) continue;
        Mat Lk = from_interleaved(m.jump_op.data() + q * 8, 2);
        Mat LdL = mul(dagger(Lk), Lk);
        Mat term = (m.jump_site[q] == b) ? kron(LdL, I2) : kron(I2, LdL);
        h = add(h, term, cd(0, -0.5 * w * m.gamma[q]));
    }
    return h;
}

Mat liouv_bond(const TnModelHost& m, int b) {
    Mat h = from_interleaved(m.h_bond.data() + (size_t)b * 32, 4);
    Mat I4 = eye(4), I2 = eye(2);
    // basis ((n_b n_{b+1}), (n'_b n'_{b+1}))
    Mat ell = scal(add(kron(h, I4), kron(I4, transpose(h)), -1.0), cd(0, -1));
    for (size_t q = 0; q < m.jump_site.size(); ++q) {
        double w = bond_share(m.L, m.jump_site[q], b);
        if (w == 0.0) continue;
        Mat Lk = from_interleaved(m.jump_op.data() + q * 8, 2);
        Mat Lb = (m.jump_site[q] == b) ? kron(Lk, I2) : kron(I2, Lk);
        Mat LdL = mul(dagger(Lb), Lb);
        Mat D = add(add(kron(Lb, conjm(Lb)), kron(LdL, I4), -0.5), kron(I4, transpose(LdL)), -0.5);
        ell = add(ell, D, w * m.gamma[q]);
    }
    // permute (n_b, n_{b+1}, n'_b, n'_{b+1}) -> (n_b, n'_b, n_{b+1}, n'_{b+1})
    Mat out(16);
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            int rn = r >> 3 & 1, rn1 = r >> 2 & 1, rp = r >> 1 & 1, rp1 = r & 1;
            int cn = c >> 3 & 1, cn1 = c >> 2 & 1, cp = c >> 1 & 1, cp1 = c & 1;
            int R = (rn << 3) | (rp << 2) | (rn1 << 1) | rp1;
            int C = (cn << 3) | (cp << 2) | (cn1 << 1) | cp1;
            out(R, C) = ell(r, c);
        }
    return out;
}

}  // namespace

// kind 0 (MPS) / 2 (PURIFIED): 4x4 exp(-i h^eff tau); kind 1 (MPDO): 16x16 exp(l tau)
std::vector<double> build_bond_gate(int kind, const TnModelHost& m, int b, double tau) {
    Mat G;
    if (kind == 1) G = expm(scal(liouv_bond(m, b), cd(tau, 0)));
    else G = expm(scal(heff_bond(m, b), cd(0, -tau)));
    std::vector<double> out(2 * G.a.size());
    for (size_t i = 0; i < G.a.size(); ++i) {
        out[2 * i] = G.a[i].real();
        out[2 * i + 1] = G.a[i].imag();
    }
    return out;
}

// embed a 4x4 gate on (n_b, n_{b+1}) into p = n*dk + k on both sites (identity on the Kraus indices)
std::vector<double> embed_purified(const std::vector<double>& g4, int dkl, int dkr) {
    const int dl = 2 * dkl, dr = 2 * dkr, D = dl * dr;
    std::vector<double> out(2 * (size_t)D * D, 0.0);
    for (int k1 = 0; k1 < dkl; ++k1)
        for (int k2 = 0; k2 < dkr; ++k2)
            for (int a = 0; a < 2; ++a)
                for (int bb = 0; bb < 2; ++bb)
                    for (int c = 0; c < 2; ++c)
                        for (int e = 0; e < 2; ++e) {
                            int row = (a * dkl + k1) * dr + (bb * dkr + k2);
                            int col = (c * dkl + k1) * dr + (e * dkr + k2);
                            int gi = (a * 2 + bb) * 4 + (c * 2 + e);
                            out[2 * ((size_t)row * D + col)] = g4[2 * gi];
                            out[2 * ((size_t)row * D + col) + 1] = g4[2 * gi + 1];
                        }
    return out;
}
