// Shared device/host helpers for the TEBD-Lindblad HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

// ---------------------------------------------------------------- complex math
template <class R> struct cplx_of;
template <> struct cplx_of<float>  { typedef float2  type; };
template <> struct cplx_of<double> { typedef double2 type; };

template <class C> struct real_of;
template <> struct real_of<float2>  { typedef float  type; };
template <> struct real_of<double2> { typedef double type; };

__host__ __device__ __forceinline__ double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ __forceinline__ float2  mkf(float a, float b) { return make_float2(a, b); }

template <class C> __host__ __device__ __forceinline__ C czero() { C z; z.x = 0; z.y = 0; return z; }

template <class C> __host__ __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <class C> __host__ __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <class C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
    C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <class C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
    C r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <class C> __host__ __device__ __forceinline__ C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
template <class C, class R> __host__ __device__ __forceinline__ C cscale(C a, R s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
// acc += a * b
template <class C> __host__ __device__ __forceinline__ void cfma(C& acc, C a, C b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <class C> __host__ __device__ __forceinline__ void cfmac(C& acc, C a, C b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
template <class To, class From> __host__ __device__ __forceinline__ To cconv(From a) { To r; r.x = a.x; r.y = a.y; return r; }

// ---------------------------------------------------------------- error codes
#define TN_OK        0
#define TN_EINVAL   -1
#define TN_ENOMEM   -2
#define TN_EHIP     -3
#define TN_ENOCONV  -4
#define TN_ENUMERIC -5

// Per-item status flags written by kernels (OR-ed into a device word).
#define TN_FLAG_NOCONV  1
#define TN_FLAG_LOGFULL 2
#define TN_FLAG_NAN     4
#define TN_FLAG_JACOBI  8   // one-sided Jacobi refinement did not converge

// ---------------------------------------------------------------- device view of a state
// Everything a kernel needs to locate tensors, bond weights and dimensions of
// instance b, plus the per-item workspace of the current chunk.
struct DevState {
    int kind;          // TN_KIND_*
    int L, B, chi, dmax;
    size_t site_cap;   // complex elements per site slot = chi * dmax * chi
    void* tens;        // B * L * site_cap elements (float2 or double2)
    double* lam;       // B * (L-1) * chi
    int* dims;         // B * (L+1)
    double* lognorm;   // B
    double* trunc;     // B
    const int* dsite;  // L physical dimensions
    double cutoff2;    // (sv_cutoff)^2, applied to Gram eigenvalues
};

// Workspace of one chunk of two-site updates (slot j for the j-th item of the chunk).
struct DevWork {
    int item0, nitems;           // first item index (within the bucket when bonds != null), items in chunk
    int parity, nb;              // layer parity and bonds per instance in this layer
    const int* bonds;            // bucket: its bond positions t (bond = parity + 2 t), bond-major items
    int bsz;                     // instances per bond position in a bucket (the batch)
    const unsigned char* mask;   // B bytes or null
    const double2* gates;        // gate table for this layer: [bond] stride gstride
    int gstride;
    int mmax, nmax;              // max Theta rows / cols
    size_t theta_stride;         // elements per item
    void* theta;                 // items * theta_stride complex128 (Theta~)
    int theta64;                 // 1: Theta~ contracted on the FP64 matrix cores (always in FP64 mode)
    double2* gram;               // items * nmax * nmax
    double2* refl;               // items * nmax * nmax   (Householder vectors)
    double2* tau;                // items * nmax
    double* dd;                  // items * nmax   (diagonal, then eigenvalues)
    double* ee;                  // items * nmax
    int logcap;                  // rotation log capacity per item
    int* logi;                   // items * logcap
    double2* logcs;              // items * logcap  (c, s)
    int* nrot;                   // items
    int* sel;                    // items * nmax  selected eigenvalue indices (descending)
    int* kout;                   // items  new bond dimension
    double* sout;                // items  kept norm s
    double* wout;                // items  discarded weight
    double2* V;                  // items * nmax * vld  (row-major n x k, leading dimension vld)
    int vld;                     // chi, or nmax when every eigenvector is formed (Jacobi refinement)
    double2* zscratch;           // items * nmax * vld  (global eigenvector scratch, large n)
    double2* pscratch;           // items * nmax*(nmax+1)/2 (packed matrix for large n)
    int* flags;                  // 1 word
    unsigned long long* counters;  // [0] items sent to the logged-QL fallback, [1] items re-orthogonalized
    int* gsz;                    // items  size of the Hermitian eigenproblem (n, or m on the QR route)
    double2* qra;                // items * nmax * nmax  Householder QR of Theta^+ (FP64 mode, wide items)
    double2* qtau;               // items * nmax
    int qr_route;                // 1: wide items (m < n) take the QR route (FP64 mode)
    int jacobi;                  // 1: one-sided Jacobi refinement of the SVD (FP64 mode)
    double* lsel;                // items * nmax  selected eigenvalues, descending (bisection path)
    int* fb;                     // items  1: item takes the logged-QL eigenvector path, or null
    int hvar;                    // Householder kernel for n <= 128: 0 MFMA block columns, 1 wave tiles
    double2* Y;                  // items * ysz  Y = Theta~ V, column-major m x r (aliases the Gram slot)
    int ldy;                     // leading dimension of Y (>= mmax)
    size_t ysz;                  // elements per item
    // sequential sweep (orthogonality centre inside the block): no Lambda_{bond-1} weights;
    // rmove: the centre leaves on site bond+1 (B_bond left-isometric, B_{bond+1} = diag(Lambda) V^+);
    // skip_gate: identity gate (centre shift)
    int unitw = 0, rmove = 0, skip_gate = 0;
};

// item -> (instance, bond); returns false for masked items
__device__ __forceinline__ bool item_coords(const DevWork& w, int j, int& b, int& bond) {
    const int g = w.item0 + j;
    if (w.bonds) {
        // a bucket's items: every instance of its first bond position, then of the next, ...
        b = g % w.bsz;
        bond = w.parity + 2 * w.bonds[g / w.bsz];
    } else {
        b = g / w.nb;
        bond = w.parity + 2 * (g % w.nb);
    }
    if (w.mask && w.mask[b]) return false;
    return true;
}

template <class T> __device__ __forceinline__ T* site_ptr(const DevState& s, int b, int i) {
    return reinterpret_cast<T*>(s.tens) + ((size_t)b * s.L + i) * s.site_cap;
}
__device__ __forceinline__ int bond_dim(const DevState& s, int b, int k) { return s.dims[(size_t)b * (s.L + 1) + k]; }
__device__ __forceinline__ double* lam_ptr(const DevState& s, int b, int bond) {
    return s.lam + ((size_t)b * (s.L - 1) + bond) * s.chi;
}
