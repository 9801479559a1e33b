// C ABI of the batched TEBD-Lindblad library: state allocation inside a
// caller-owned device arena, Trotter layer scheduling in chunks of independent
// two-site updates, dissipative steps, measurement, state I/O and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tebd.h"
#include "common.h"
#include "host_gates.h"
#include "launch.h"

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(TN_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ profiling
void prof_begin(Prof* p, int id, hipStream_t st) {
    if (!p || !p->on) return;
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, st);
    p->open[id] = e;
}
void prof_end(Prof* p, int id, hipStream_t st) {
    if (!p || !p->on || !p->open[id]) return;
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, st);
    p->ev[id].push_back(std::make_pair(p->open[id], e));
    p->open[id] = nullptr;
}

// ------------------------------------------------------------------ state
struct Layout {
    size_t off_tens, off_lam, off_dims, off_lognorm, off_trunc, off_dsite, off_mask, off_jumped, off_glog, off_gwt,
        off_gates, off_rnd, off_vals, off_lval, off_nrm, off_jsite, off_jop, off_jLdL, off_gam, off_ceach, off_cmean, off_cvar,
        off_flags, off_bkt, off_ws;
    size_t ws_bytes, total;
    // workspace sub-layout (update)
    size_t u_theta, u_gram, u_refl, u_tau, u_dd, u_ee, u_logi, u_logcs, u_nrot, u_sel, u_kout, u_sout, u_wout, u_V,
        u_z, u_p, u_gsz, u_qra, u_qtau, u_lsel, u_fb, u_bytes;
    // workspace sub-layout (measurement)
    size_t m_R, m_E, m_X, m_Y, m_W, m_bytes;
};

struct tn_state {
    int kind, L, B, chi, chik, prec, dmax, njump;
    int chunk, nbm, mmax, nmax, logcap, gstride, nbmax;
    // largest m = d_b D_b and Gram order n = d_{b+1} D_{b+2} over all bonds, D the largest bond
    // dimensions the chain allows (mmax, nmax: the workspace bounds d_max chi)
    int mstruct = 1, nstruct = 1;
    double cutoff;
    std::vector<int> dsite;
    TnModelHost model;
    hipStream_t stream;
    char* arena;
    Layout lay;
    size_t site_cap, esz;
    // gate cache: tau -> slot
    double slot_tau[2];
    bool slot_valid[2];
    Prof prof;
    // one captured Trotter step (all layers, unmasked) per schedule and order, replayed by tebd_step
    hipGraphExec_t gexec[2][3][2] = {};  // [schedule][order][masked]
    int schedule = TN_SCHED_LAYER;
    int use_graph = 1;
    // autotuner: Householder variant for n <= 128 chosen by timing on the state's own data
    int tuned = 0;
    int hvar = 0;
    float tune_ms[2] = {0.0f, 0.0f};
    // chunks of one layer alternate between `stream` and `aux` (a stream the library owns, default
    // priority), each with its own workspace slot, so that kernels of different chunks can share
    // the compute units; joined back into `stream` before the layer's reduction
    int nslots = 1;
    int overlap = 1;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    Prof prof2;  // timing of the work launched on aux
    // asynchronous measurement: a caller-owned second buffer holds a snapshot of the state
    // (tensors, weights, dims, log-norms, copied in stream order) and the measurement's own
    // workspace and outputs; the measurement runs on `mstream` while later steps run on `stream`
    char* abuf = nullptr;
    size_t a_snap = 0, a_nrm = 0, a_ceach = 0, a_cmean = 0, a_cvar = 0, a_ws = 0, a_total = 0;
    hipStream_t mstream = nullptr;
    hipEvent_t ev_snap = nullptr;
    bool apending = false;
    Prof prof3;  // timing of the work launched on mstream
    // this device's address of the static measurement scratch (measure_corr_noalloc)
    char* scratch = nullptr;
    // split mode: Theta formation on the FP64 matrix cores instead of the FP32 ones
    int theta64 = 0;
    // bond-size buckets: the bond positions t of each parity grouped by the order their Gram
    // matrices can reach (structural bond dimensions), largest class first; a chunk holds items
    // of one bucket, sized and dispatched for that bucket's largest shape, with the Householder
    // variant the autotuner chose for its class
    struct Bucket {
        int start, count, nmax, mmax, hvar;
        float tune_ms[2];
    };
    std::vector<Bucket> bk[2];
    int bucketing = 1;
    int ncu = 256;  // compute units of the arena's device: the smallest layer that is bucketed
    ~tn_state() {
        for (hipStream_t q : {aux, mstream})
            if (q) {
                hipStreamSynchronize(q);
                hipStreamDestroy(q);
            }
        for (hipEvent_t e : {ev_fork, ev_join, ev_snap})
            if (e) hipEventDestroy(e);
    }
};

// workspace slots: two when a layer can span more than one chunk
static int workspace_slots(int L, int B, int chunk) {
    const long items = (long)B * ((L - 1 + 1) / 2);
    return items > chunk ? 2 : 1;
}

static void drop_graphs(tn_state* s) {
    for (int sc = 0; sc < 2; ++sc)
        for (int o = 0; o < 3; ++o)
            for (int m = 0; m < 2; ++m)
                if (s->gexec[sc][o][m]) {
                    hipGraphExecDestroy(s->gexec[sc][o][m]);
                    s->gexec[sc][o][m] = nullptr;
                }
}

static inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static int physical_dims(int kind, int L, int chik, const std::vector<int>& jsite, std::vector<int>& d) {
    d.assign(L, 2);
    if (kind == TN_KIND_MPDO) d.assign(L, 4);
    if (kind == TN_KIND_PURIFIED)
        for (int s : jsite) d[s] = 2 * chik;
    return 0;
}

// measurement workspace of a group of nbm instances (right environments, left strings and the
// GEMM temporaries of the sweep); sets ly.m_* and returns ly.m_bytes
static size_t meas_sublayout(Layout& ly, int L, int chi, int dmax, size_t esz, int nbm) {
    size_t m = 0;
    size_t cc = (size_t)chi * chi;
    ly.m_R = m; m = al(m + std::max((size_t)(L + 1) * nbm * cc * esz, (size_t)nbm * (L + 1) * chi * 16));
    ly.m_E = m; m = al(m + std::max((size_t)nbm * cc * esz, (size_t)nbm * (L + 1) * chi * 16));
    ly.m_X = m; m = al(m + (size_t)nbm * L * cc * esz);
    ly.m_Y = m; m = al(m + (size_t)nbm * L * chi * dmax * chi * esz);
    ly.m_W = m; m = al(m + (size_t)nbm * chi * dmax * chi * esz);
    ly.m_bytes = m;
    return m;
}

static void compute_layout(Layout& ly, int kind, int L, int B, int chi, int dmax, int prec, int chunk, int nbm,
                           int njump, int logcap, int nslots) {
    const size_t esz = prec == 0 ? 16 : 8;
    const size_t site_cap = (size_t)chi * dmax * chi;
    const int mmax = chi * dmax, nmax = dmax * chi;
    const int nbmax = (L - 1 + 1) / 2;
    size_t o = 0;
    ly.off_tens = o; o = al(o + (size_t)B * L * site_cap * esz);
    ly.off_lam = o; o = al(o + (size_t)B * (L - 1) * chi * 8);
    ly.off_dims = o; o = al(o + (size_t)B * (L + 1) * 4);
    ly.off_lognorm = o; o = al(o + (size_t)B * 8);
    ly.off_trunc = o; o = al(o + (size_t)B * 8);
    ly.off_dsite = o; o = al(o + (size_t)L * 4);
    ly.off_mask = o; o = al(o + (size_t)B);
    ly.off_jumped = o; o = al(o + (size_t)B * 4);
    ly.off_glog = o; o = al(o + (size_t)B * nbmax * 8);
    ly.off_gwt = o; o = al(o + (size_t)B * nbmax * 8);
    ly.off_gates = o; o = al(o + (size_t)2 * (L - 1) * 256 * 16);
    ly.off_rnd = o; o = al(o + (size_t)B * (njump > 0 ? njump : 1) * 2 * 8);
    ly.off_vals = o; o = al(o + (size_t)B * (njump > 0 ? njump : 1) * 8);
    ly.off_lval = o; o = al(o + (size_t)B * (njump > 0 ? njump : 1) * 16);
    ly.off_nrm = o; o = al(o + (size_t)B * 8);
    ly.off_jsite = o; o = al(o + (size_t)TN_MAX_JUMPS * 4);
    ly.off_jop = o; o = al(o + (size_t)TN_MAX_JUMPS * 4 * 16);
    ly.off_jLdL = o; o = al(o + (size_t)TN_MAX_JUMPS * 4 * 16);
    ly.off_gam = o; o = al(o + (size_t)TN_MAX_JUMPS * 8);
    ly.off_ceach = o; o = al(o + (size_t)B * L * L * 16);
    ly.off_cmean = o; o = al(o + (size_t)L * L * 16);
    ly.off_cvar = o; o = al(o + (size_t)L * L * 8);
    ly.off_flags = o; o = al(o + 64);
    ly.off_bkt = o; o = al(o + (size_t)2 * nbmax * 4);
    ly.off_ws = o;
    // update workspace
    size_t u = 0;
    // Theta~ in complex128 in both precisions
    ly.u_theta = u; u = al(u + (size_t)chunk * mmax * nmax * 16);
    ly.u_gram = u; u = al(u + (size_t)chunk * nmax * nmax * 16);
    ly.u_refl = u; u = al(u + (size_t)chunk * nmax * nmax * 16);
    ly.u_tau = u; u = al(u + (size_t)chunk * nmax * 16);
    ly.u_dd = u; u = al(u + (size_t)chunk * nmax * 8);
    ly.u_ee = u; u = al(u + (size_t)chunk * nmax * 8);
    ly.u_logi = u; u = al(u + (size_t)chunk * logcap * 4);
    ly.u_logcs = u; u = al(u + (size_t)chunk * logcap * 16);
    ly.u_nrot = u; u = al(u + (size_t)chunk * 4);
    ly.u_sel = u; u = al(u + (size_t)chunk * nmax * 4);
    ly.u_kout = u; u = al(u + (size_t)chunk * 4);
    ly.u_sout = u; u = al(u + (size_t)chunk * 8);
    ly.u_wout = u; u = al(u + (size_t)chunk * 8);
    // FP64 mode forms every eigenvector (Jacobi refinement): V is n x n there, n x chi otherwise
    const size_t vld = prec == 0 ? (size_t)nmax : (size_t)chi;
    ly.u_V = u; u = al(u + (size_t)chunk * nmax * vld * 16);
    ly.u_z = u; if ((size_t)nmax * vld > 8192) u = al(u + (size_t)chunk * nmax * vld * 16);
    ly.u_p = u; if (nmax > 128) u = al(u + (size_t)chunk * ((size_t)nmax * (nmax + 1) / 2) * 16);
    ly.u_gsz = u; u = al(u + (size_t)chunk * 4);
    ly.u_qra = u; if (prec == 0) u = al(u + (size_t)chunk * nmax * nmax * 16);
    ly.u_qtau = u; if (prec == 0) u = al(u + (size_t)chunk * nmax * 16);
    ly.u_lsel = u; u = al(u + (size_t)chunk * nmax * 8);
    ly.u_fb = u; u = al(u + (size_t)chunk * 4);
    ly.u_bytes = u;
    meas_sublayout(ly, L, chi, dmax, esz, nbm);
    ly.ws_bytes = std::max((size_t)nslots * ly.u_bytes, ly.m_bytes);
    ly.total = ly.off_ws + ly.ws_bytes;
    (void)kind;
}

static int default_chunk(int L, int B, int chi, int dmax) {
    const int nbmax = (L - 1 + 1) / 2;
    long items = (long)B * nbmax;
    int n = chi * dmax;
    long cap = n <= 128 ? 8192 : (n <= 256 ? 1024 : 64);
    return (int)std::max(1L, std::min(items, cap));
}
static int default_nbm(int B, int L, int chi) {
    long per = (long)L * chi * chi;
    long cap = std::max(1L, (long)(64L * 1024 * 1024 * 4) / std::max(1L, per));
    return (int)std::max(1L, std::min((long)B, std::min(cap, 1024L)));
}
static int log_capacity(int nmax) { return std::max(64, 4 * nmax * nmax); }

static bool model_ok(const tn_model* m, std::string& why) {
    if (!m) { why = "model is null"; return false; }
    if (m->L < 2) { why = "L must be >= 2"; return false; }
    if (m->d != 2) { why = "local dimension d must be 2"; return false; }
    if (!m->h_bond) { why = "h_bond is null"; return false; }
    if (m->n_jumps < 0 || m->n_jumps > TN_MAX_JUMPS) { why = "n_jumps must be in 0..256"; return false; }
    if (m->n_jumps > 0 && (!m->jump_site || !m->jump_op || !m->gamma)) { why = "jump arrays are null"; return false; }
    for (int q = 0; q < m->n_jumps; ++q) {
        if (m->jump_site[q] < 0 || m->jump_site[q] >= m->L) { why = "jump site out of range"; return false; }
        if (!(m->gamma[q] >= 0) || !std::isfinite(m->gamma[q])) { why = "rate negative or not finite"; return false; }
        for (int e = 0; e < 8; ++e)
            if (!std::isfinite(m->jump_op[8 * q + e])) { why = "jump operator not finite"; return false; }
    }
    for (size_t e = 0; e < (size_t)(m->L - 1) * 32; ++e)
        if (!std::isfinite(m->h_bond[e])) { why = "h_bond not finite"; return false; }
    return true;
}

extern "C" size_t mps_arena_bytes(int kind, int L, int batch, int chi_max, int chi_k_max, int precision,
                                  int chunk_items) {
    if (L < 2 || batch < 1 || chi_max < 1 || (precision != 0 && precision != 1)) return 0;
    if (kind < 0 || kind > 2) return 0;
    int dmax = kind == TN_KIND_MPDO ? 4 : (kind == TN_KIND_PURIFIED ? 2 * std::max(1, chi_k_max) : 2);
    int chunk = chunk_items > 0 ? chunk_items : default_chunk(L, batch, chi_max, dmax);
    int nbm = default_nbm(batch, L, chi_max);
    Layout ly;
    compute_layout(ly, kind, L, batch, chi_max, dmax, precision, chunk, nbm, TN_MAX_JUMPS,
                   log_capacity(std::min(dmax * chi_max, 512)),
                   workspace_slots(L, batch, chunk));
    return ly.total;
}

template <class T>
static inline T* at(tn_state* s, size_t off) { return reinterpret_cast<T*>(s->arena + off); }

static DevState dev_state(tn_state* s) {
    DevState d;
    d.kind = s->kind;
    d.L = s->L;
    d.B = s->B;
    d.chi = s->chi;
    d.dmax = s->dmax;
    d.site_cap = s->site_cap;
    d.tens = s->arena + s->lay.off_tens;
    d.lam = at<double>(s, s->lay.off_lam);
    d.dims = at<int>(s, s->lay.off_dims);
    d.lognorm = at<double>(s, s->lay.off_lognorm);
    d.trunc = at<double>(s, s->lay.off_trunc);
    d.dsite = at<int>(s, s->lay.off_dsite);
    d.cutoff2 = s->cutoff * s->cutoff;
    return d;
}

// packed host layout of one instance
static size_t packed_tensor_elems(const tn_state* s, const int* dims) {
    size_t n = 0;
    for (int i = 0; i < s->L; ++i) n += (size_t)dims[i] * s->dsite[i] * dims[i + 1];
    return n;
}

// largest bond dimensions D_0 .. D_L an open chain with local dimensions d allows under chi
static std::vector<double> structural_dims(const std::vector<int>& d, int chi) {
    const int L = (int)d.size();
    std::vector<double> D(L + 1, 1.0);
    double left = 1.0;
    for (int b = 1; b < L; ++b) {
        left *= d[b - 1];
        double right = 1.0;
        for (int i = b; i < L && right < 4096.0; ++i) right *= d[i];
        D[b] = std::min<double>(chi, std::min(left, right));
    }
    return D;
}

// size class of a Gram order: the boundaries at which the update kernels change
static int size_class(int n) { return n <= 64 ? 0 : (n <= 128 ? 1 : (n <= 256 ? 2 : 3)); }

// the buckets of both parities (host side) and their bond-position table (device side)
static int build_buckets(tn_state* s) {
    const std::vector<double> D = structural_dims(s->dsite, s->chi);
    std::vector<int> table((size_t)2 * s->nbmax, 0);
    for (int p = 0; p < 2; ++p) {
        s->bk[p].clear();
        const int nb = p <= s->L - 2 ? ((s->L - 2 - p) / 2 + 1) : 0;
        int pos = 0;
        for (int c = 3; c >= 0; --c) {
            tn_state::Bucket bkt{pos, 0, 0, 0, s->hvar, {0.0f, 0.0f}};
            for (int t = 0; t < nb; ++t) {
                const int bond = p + 2 * t;
                const int n = (int)(s->dsite[bond + 1] * D[bond + 2]), m = (int)(s->dsite[bond] * D[bond]);
                if (size_class(n) != c) continue;
                table[(size_t)p * s->nbmax + pos++] = t;
                bkt.count++;
                bkt.nmax = std::max(bkt.nmax, n);
                bkt.mmax = std::max(bkt.mmax, m);
                s->nstruct = std::max(s->nstruct, n);
                s->mstruct = std::max(s->mstruct, m);
            }
            if (bkt.count) s->bk[p].push_back(bkt);
        }
    }
    HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_bkt, table.data(), table.size() * 4, hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TN_OK;
}

extern "C" int mps_set_instance(void* h, int inst, const int* dims, const double* tensors, const double* lambdas,
                                double lognorm);
extern "C" int mps_replicate(void* h, int src);

// ------------------------------------------------------------------ static measurement scratch
// The workspace of measure_corr_noalloc: a file-scope device array that every GPU the library
// runs on holds, at its own address, until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with that device current, kept in g_scratch, and used
// from then on.
static __device__ __align__(256) char scratch[TN_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch;

static int scratch_setup(int dev, char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return TN_OK;
    }
    int prev = -1;
    HIPCHK(hipGetDevice(&prev));
    if (prev != dev) HIPCHK(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != dev) HIPCHK(hipSetDevice(prev));
    if (e != hipSuccess || !ptr)
        return fail(TN_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = reinterpret_cast<char*>(ptr);
    *out = reinterpret_cast<char*>(ptr);
    return TN_OK;
}

extern "C" int mps_alloc(void** out, int kind, const tn_model* model, int batch, int chi_max, int chi_k_max,
                         int precision, const int* init_occ, double sv_cutoff, void* arena, size_t arena_bytes,
                         void* hip_stream) {
    g_err.clear();
    if (!out) return fail(TN_EINVAL, "out is null");
    *out = nullptr;
    std::string why;
    if (!model_ok(model, why)) return fail(TN_EINVAL, why);
    if (kind < 0 || kind > 2) return fail(TN_EINVAL, "unknown kind");
    if (batch < 1 || chi_max < 1) return fail(TN_EINVAL, "batch and chi_max must be >= 1");
    if (chi_max > 256) return fail(TN_EINVAL, "chi_max must be <= 256");
    if (precision != 0 && precision != 1) return fail(TN_EINVAL, "precision must be TN_FP64 or TN_SPLIT");
    if (!init_occ) return fail(TN_EINVAL, "init_occ is null");
    if (!arena) return fail(TN_EINVAL, "arena is null");
    if (!(sv_cutoff >= 0.0 && sv_cutoff < 1.0)) return fail(TN_EINVAL, "sv_cutoff must be in [0, 1)");
    if (kind == TN_KIND_PURIFIED && (chi_k_max < 1 || chi_k_max > 4))
        return fail(TN_EINVAL, "chi_k_max must be in 1..4");
    const int L = model->L;
    for (int i = 0; i < L; ++i)
        if (init_occ[i] != 0 && init_occ[i] != 1) return fail(TN_EINVAL, "init_occ entries must be 0 or 1");
    tn_state* s = new tn_state();
    s->kind = kind;
    s->L = L;
    s->B = batch;
    s->chi = chi_max;
    s->chik = kind == TN_KIND_PURIFIED ? chi_k_max : 1;
    s->prec = precision;
    s->cutoff = sv_cutoff;
    s->njump = model->n_jumps;
    s->model.L = L;
    s->model.h_bond.assign(model->h_bond, model->h_bond + (size_t)(L - 1) * 32);
    for (int q = 0; q < model->n_jumps; ++q) {
        s->model.jump_site.push_back(model->jump_site[q]);
        s->model.gamma.push_back(model->gamma[q]);
        for (int e = 0; e < 8; ++e) s->model.jump_op.push_back(model->jump_op[8 * q + e]);
    }
    physical_dims(kind, L, s->chik, s->model.jump_site, s->dsite);
    s->dmax = *std::max_element(s->dsite.begin(), s->dsite.end());
    for (int b = 0; b + 1 < L; ++b)
        if (s->dsite[b] * s->dsite[b + 1] > 16) {
            delete s;
            return fail(TN_EINVAL, "bond physical dimension d_b*d_{b+1} exceeds 16 (adjacent purified jump sites)");
        }
    {
        // Theta of bond b is (d_b D_b) x (d_{b+1} D_{b+2}) with D the largest bond dimensions the
        // chain allows under chi_max.  The eigenproblem is the Gram matrix of order n = d_{b+1}
        // D_{b+2} (split mode), or of order min(m, n) in FP64 mode, where wide Theta takes the QR
        // route; it must stay <= 512, and Theta's sides <= 1024.
        const std::vector<double> D = structural_dims(s->dsite, chi_max);
        int worst = 0, side = 0;
        for (int b = 0; b + 1 < L; ++b) {
            const int m = (int)(s->dsite[b] * D[b]), n = (int)(s->dsite[b + 1] * D[b + 2]);
            worst = std::max(worst, precision == 0 ? std::min(m, n) : n);
            side = std::max(side, std::max(m, n));
        }
        if (worst > 512 || side > 1024) {
            delete s;
            return fail(TN_EINVAL, precision == 0
                                       ? "a bond's eigenproblem order min(m, n) would exceed 512 (or a side of Theta 1024)"
                                       : "a bond's Gram order d chi_r would exceed 512 in split mode");
        }
    }
    s->site_cap = (size_t)chi_max * s->dmax * chi_max;
    s->esz = precision == 0 ? 16 : 8;
    s->mmax = chi_max * s->dmax;
    s->nmax = s->dmax * chi_max;
    s->chunk = default_chunk(L, batch, chi_max, s->dmax);
    s->nbm = default_nbm(batch, L, chi_max);
    s->logcap = log_capacity(std::min(s->nmax, 512));
    s->gstride = 256;
    s->nbmax = (L - 1 + 1) / 2;
    s->nslots = workspace_slots(L, batch, s->chunk);
    compute_layout(s->lay, kind, L, batch, chi_max, s->dmax, precision, s->chunk, s->nbm, TN_MAX_JUMPS, s->logcap,
                   s->nslots);
    if (arena_bytes < s->lay.total) {
        size_t need = s->lay.total;
        delete s;
        char buf[128];
        snprintf(buf, sizeof buf, "arena too small: need %zu bytes", need);
        return fail(TN_ENOMEM, buf);
    }
    s->arena = reinterpret_cast<char*>(arena);
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    {
        // the arena's device holds this state; its copy of the static scratch is looked up now
        int dev = -1;
        hipPointerAttribute_t pa;
        if (hipPointerGetAttributes(&pa, arena) == hipSuccess && pa.device >= 0) dev = pa.device;
        else if (hipGetDevice(&dev) != hipSuccess) dev = -1;
        const int rc0 = dev < 0 ? fail(TN_EHIP, "cannot tell the arena's device") : scratch_setup(dev, &s->scratch);
        if (rc0 != TN_OK) {
            delete s;
            return rc0;
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            s->ncu = ncu;
    }
    if (s->nslots == 2) {
        bool ok = hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking) == hipSuccess;
        for (hipEvent_t* e : {&s->ev_fork, &s->ev_join})
            ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            delete s;
            return fail(TN_EHIP, "creating the second stream or its events failed");
        }
    }
    s->slot_valid[0] = s->slot_valid[1] = false;
    {
        const int rcb = build_buckets(s);
        if (rcb != TN_OK) {
            delete s;
            return rcb;
        }
    }
    // constant tables
    int rc;
    {
        hipError_t e = hipMemcpyAsync(s->arena + s->lay.off_dsite, s->dsite.data(), L * sizeof(int),
                                      hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) { delete s; return fail(TN_EHIP, hipGetErrorString(e)); }
        std::vector<int> js(s->model.jump_site);
        std::vector<double2> jo, jl;
        for (int q = 0; q < s->njump; ++q) {
            double2 o[4];
            for (int e2 = 0; e2 < 4; ++e2) o[e2] = mk(s->model.jump_op[8 * q + 2 * e2], s->model.jump_op[8 * q + 2 * e2 + 1]);
            for (int e2 = 0; e2 < 4; ++e2) jo.push_back(o[e2]);
            // L^+ L
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) {
                    double2 acc = mk(0, 0);
                    for (int k = 0; k < 2; ++k) cfmac(acc, o[k * 2 + r], o[k * 2 + c]);
                    jl.push_back(acc);
                }
        }
        if (s->njump) {
            hipMemcpyAsync(s->arena + s->lay.off_jsite, js.data(), js.size() * 4, hipMemcpyHostToDevice, s->stream);
            hipMemcpyAsync(s->arena + s->lay.off_jop, jo.data(), jo.size() * 16, hipMemcpyHostToDevice, s->stream);
            hipMemcpyAsync(s->arena + s->lay.off_jLdL, jl.data(), jl.size() * 16, hipMemcpyHostToDevice, s->stream);
            hipMemcpyAsync(s->arena + s->lay.off_gam, s->model.gamma.data(), s->njump * 8, hipMemcpyHostToDevice,
                           s->stream);
        }
        hipMemsetAsync(s->arena + s->lay.off_flags, 0, 64, s->stream);
        hipMemsetAsync(s->arena + s->lay.off_mask, 0, (size_t)batch, s->stream);
    }
    // product state, instance 0, then replicate
    std::vector<int> dims(L + 1, 1);
    std::vector<double> tens;
    for (int i = 0; i < L; ++i) {
        int d = s->dsite[i];
        std::vector<double> t(2 * d, 0.0);
        int p;
        if (kind == TN_KIND_MPS) p = init_occ[i];
        else if (kind == TN_KIND_MPDO) p = 3 * init_occ[i];
        else p = init_occ[i] * (d / 2);
        t[2 * p] = 1.0;
        tens.insert(tens.end(), t.begin(), t.end());
    }
    std::vector<double> lams(L - 1, 1.0);
    rc = mps_set_instance(s, 0, dims.data(), tens.data(), lams.data(), 0.0);
    if (rc) { delete s; return rc; }
    rc = mps_replicate(s, 0);
    if (rc) { delete s; return rc; }
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { delete s; return fail(TN_EHIP, hipGetErrorString(e)); }
    *out = s;
    return TN_OK;
}

extern "C" int mps_free(void* h) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    hipStreamSynchronize(s->stream);
    if (s->mstream) hipStreamSynchronize(s->mstream);
    for (Prof* p : {&s->prof, &s->prof2, &s->prof3})
        for (int k = 0; k < TN_K_COUNT; ++k)
            for (auto& pr : p->ev[k]) {
                hipEventDestroy(pr.first);
                hipEventDestroy(pr.second);
            }
    if (s->prof.ref) hipEventDestroy(s->prof.ref);
    drop_graphs(s);
    delete s;
    return TN_OK;
}

extern "C" const char* mps_last_error(void) { return g_err.c_str(); }

extern "C" size_t mps_instance_tensor_capacity(const void* h) {
    const tn_state* s = reinterpret_cast<const tn_state*>(h);
    return s ? (size_t)s->L * s->site_cap : 0;
}
extern "C" size_t mps_instance_lambda_capacity(const void* h) {
    const tn_state* s = reinterpret_cast<const tn_state*>(h);
    return s ? (size_t)(s->L - 1) * s->chi : 0;
}

extern "C" int mps_set_instance(void* h, int inst, const int* dims, const double* tensors, const double* lambdas,
                                double lognorm) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s || !dims || !tensors || !lambdas) return fail(TN_EINVAL, "null argument");
    if (inst < 0 || inst >= s->B) return fail(TN_EINVAL, "instance out of range");
    if (dims[0] != 1 || dims[s->L] != 1) return fail(TN_EINVAL, "dims[0] and dims[L] must be 1");
    const std::vector<double> Dmax = structural_dims(s->dsite, s->chi);
    for (int i = 1; i < s->L; ++i)
        if (dims[i] < 1 || dims[i] > Dmax[i])
            return fail(TN_EINVAL, "bond dimension out of range (1 .. min(chi_max, product of the local dimensions "
                                   "on either side))");
    {
        size_t nt = 0, nl = 0;
        for (int i = 0; i < s->L; ++i) nt += (size_t)dims[i] * s->dsite[i] * dims[i + 1];
        for (int b = 1; b < s->L; ++b) nl += dims[b];
        for (size_t e = 0; e < 2 * nt; ++e)
            if (!std::isfinite(tensors[e])) return fail(TN_EINVAL, "tensor entries must be finite");
        for (size_t e = 0; e < nl; ++e)
            if (!(lambdas[e] >= 0.0) || !std::isfinite(lambdas[e]))
                return fail(TN_EINVAL, "bond weights must be finite and >= 0");
        if (!std::isfinite(lognorm)) return fail(TN_EINVAL, "lognorm must be finite");
    }
    size_t off = 0;
    for (int i = 0; i < s->L; ++i) {
        size_t ne = (size_t)dims[i] * s->dsite[i] * dims[i + 1];
        char* dst = s->arena + s->lay.off_tens + (((size_t)inst * s->L + i) * s->site_cap) * s->esz;
        if (s->prec == 0) {
            HIPCHK(hipMemcpyAsync(dst, tensors + 2 * off, ne * 16, hipMemcpyHostToDevice, s->stream));
        } else {
            std::vector<float> f(2 * ne);
            for (size_t e = 0; e < 2 * ne; ++e) f[e] = (float)tensors[2 * off + e];
            HIPCHK(hipMemcpyAsync(dst, f.data(), ne * 8, hipMemcpyHostToDevice, s->stream));
            HIPCHK(hipStreamSynchronize(s->stream));
        }
        off += ne;
    }
    std::vector<double> lam((size_t)(s->L - 1) * s->chi, 0.0);
    size_t lo = 0;
    for (int b = 0; b + 1 < s->L; ++b) {
        for (int a = 0; a < dims[b + 1]; ++a) lam[(size_t)b * s->chi + a] = lambdas[lo + a];
        lo += dims[b + 1];
    }
    HIPCHK(hipMemcpyAsync(at<double>(s, s->lay.off_lam) + (size_t)inst * (s->L - 1) * s->chi, lam.data(),
                          lam.size() * 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(at<int>(s, s->lay.off_dims) + (size_t)inst * (s->L + 1), dims, (s->L + 1) * 4,
                          hipMemcpyHostToDevice, s->stream));
    double z = 0.0;
    HIPCHK(hipMemcpyAsync(at<double>(s, s->lay.off_lognorm) + inst, &lognorm, 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(at<double>(s, s->lay.off_trunc) + inst, &z, 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TN_OK;
}

extern "C" int mps_get_instance(const void* h, int inst, int* dims, double* tensors, double* lambdas,
                                double* lognorm, double* trunc) {
    const tn_state* s = reinterpret_cast<const tn_state*>(h);
    if (!s || !dims) return fail(TN_EINVAL, "null argument");
    if (inst < 0 || inst >= s->B) return fail(TN_EINVAL, "instance out of range");
    tn_state* sm = const_cast<tn_state*>(s);
    HIPCHK(hipMemcpyAsync(dims, at<int>(sm, s->lay.off_dims) + (size_t)inst * (s->L + 1), (s->L + 1) * 4,
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (tensors) {
        size_t off = 0;
        for (int i = 0; i < s->L; ++i) {
            size_t ne = (size_t)dims[i] * s->dsite[i] * dims[i + 1];
            const char* src = s->arena + s->lay.off_tens + (((size_t)inst * s->L + i) * s->site_cap) * s->esz;
            if (s->prec == 0) {
                HIPCHK(hipMemcpyAsync(tensors + 2 * off, src, ne * 16, hipMemcpyDeviceToHost, s->stream));
            } else {
                std::vector<float> f(2 * ne);
                HIPCHK(hipMemcpyAsync(f.data(), src, ne * 8, hipMemcpyDeviceToHost, s->stream));
                HIPCHK(hipStreamSynchronize(s->stream));
                for (size_t e = 0; e < 2 * ne; ++e) tensors[2 * off + e] = f[e];
            }
            off += ne;
        }
    }
    if (lambdas) {
        std::vector<double> lam((size_t)(s->L - 1) * s->chi);
        HIPCHK(hipMemcpyAsync(lam.data(), at<double>(sm, s->lay.off_lam) + (size_t)inst * (s->L - 1) * s->chi,
                              lam.size() * 8, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        size_t lo = 0;
        for (int b = 0; b + 1 < s->L; ++b) {
            for (int a = 0; a < dims[b + 1]; ++a) lambdas[lo + a] = lam[(size_t)b * s->chi + a];
            lo += dims[b + 1];
        }
    }
    if (lognorm)
        HIPCHK(hipMemcpyAsync(lognorm, at<double>(sm, s->lay.off_lognorm) + inst, 8, hipMemcpyDeviceToHost, s->stream));
    if (trunc)
        HIPCHK(hipMemcpyAsync(trunc, at<double>(sm, s->lay.off_trunc) + inst, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TN_OK;
}

extern "C" int mps_replicate(void* h, int src) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    if (src < 0 || src >= s->B) return fail(TN_EINVAL, "instance out of range");
    const size_t tb = (size_t)s->L * s->site_cap * s->esz;
    const size_t lb = (size_t)(s->L - 1) * s->chi * 8;
    const size_t db = (size_t)(s->L + 1) * 4;
    for (int b = 0; b < s->B; ++b) {
        if (b == src) continue;
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_tens + (size_t)b * tb, s->arena + s->lay.off_tens + (size_t)src * tb,
                              tb, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_lam + (size_t)b * lb, s->arena + s->lay.off_lam + (size_t)src * lb,
                              lb, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_dims + (size_t)b * db, s->arena + s->lay.off_dims + (size_t)src * db,
                              db, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_lognorm + (size_t)b * 8, s->arena + s->lay.off_lognorm + (size_t)src * 8,
                              8, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_trunc + (size_t)b * 8, s->arena + s->lay.off_trunc + (size_t)src * 8,
                              8, hipMemcpyDeviceToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return TN_OK;
}

// ------------------------------------------------------------------ gates
static int upload_gates(tn_state* s, int slot, double tau) {
    if (s->slot_valid[slot] && s->slot_tau[slot] == tau) return TN_OK;
    std::vector<double> all((size_t)(s->L - 1) * s->gstride * 2, 0.0);
    for (int b = 0; b + 1 < s->L; ++b) {
        std::vector<double> g;
        try {
            g = build_bond_gate(s->kind == TN_KIND_MPDO ? 1 : 0, s->model, b, tau);
        } catch (const std::exception& ex) {
            return fail(TN_ENUMERIC, ex.what());
        }
        if (s->kind == TN_KIND_PURIFIED) g = embed_purified(g, s->dsite[b] / 2, s->dsite[b + 1] / 2);
        std::copy(g.begin(), g.end(), all.begin() + (size_t)b * s->gstride * 2);
    }
    HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_gates + (size_t)slot * (s->L - 1) * 256 * 16, all.data(),
                          all.size() * 8, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->slot_tau[slot] = tau;
    s->slot_valid[slot] = true;
    return TN_OK;
}

extern "C" int tn_gate(int kind, const tn_model* model, int bond, double tau, double* out) {
    std::string why;
    if (!model_ok(model, why)) return fail(TN_EINVAL, why);
    if (!out || bond < 0 || bond > model->L - 2) return fail(TN_EINVAL, "bad bond or null output");
    TnModelHost m;
    m.L = model->L;
    m.h_bond.assign(model->h_bond, model->h_bond + (size_t)(model->L - 1) * 32);
    for (int q = 0; q < model->n_jumps; ++q) {
        m.jump_site.push_back(model->jump_site[q]);
        m.gamma.push_back(model->gamma[q]);
        for (int e = 0; e < 8; ++e) m.jump_op.push_back(model->jump_op[8 * q + e]);
    }
    try {
        std::vector<double> g = build_bond_gate(kind == TN_KIND_MPDO ? 1 : 0, m, bond, tau);
        std::copy(g.begin(), g.end(), out);
    } catch (const std::exception& ex) {
        return fail(TN_ENUMERIC, ex.what());
    }
    return TN_OK;
}

// ------------------------------------------------------------------ flags
static int check_flags(tn_state* s) {
    int flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, s->arena + s->lay.off_flags, 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (flags) {
        HIPCHK(hipMemsetAsync(s->arena + s->lay.off_flags, 0, 4, s->stream));
        if (flags & TN_FLAG_NAN) return fail(TN_ENUMERIC, "NaN in a two-site update");
        if (flags & TN_FLAG_LOGFULL) return fail(TN_ENOCONV, "rotation log capacity exceeded");
        if (flags & TN_FLAG_NOCONV) return fail(TN_ENOCONV, "tridiagonal QL did not converge");
        if (flags & TN_FLAG_JACOBI) return fail(TN_ENOCONV, "one-sided Jacobi refinement did not converge");
    }
    return TN_OK;
}

// ------------------------------------------------------------------ TEBD
// workspace view of the chunk of items [i0, i0 + nitems) of one layer
static DevWork chunk_work(tn_state* s, int parity, int nb, int slot, long i0, int nitems,
                          const unsigned char* mask_dev, int wslot = 0, const tn_state::Bucket* bkt = nullptr) {
    char* ws = s->arena + s->lay.off_ws + (size_t)wslot * s->lay.u_bytes;
    DevWork w;
    w.item0 = (int)i0;
    w.nitems = nitems;
    w.parity = parity;
    w.nb = nb;
    w.bonds = bkt ? at<int>(s, s->lay.off_bkt) + (size_t)parity * s->nbmax + bkt->start : nullptr;
    w.bsz = s->B;
    w.mask = mask_dev;
    w.gates = reinterpret_cast<const double2*>(s->arena + s->lay.off_gates + (size_t)slot * (s->L - 1) * 256 * 16);
    w.gstride = s->gstride;
    // per-item strides and kernel choices follow the bucket's largest shape, or without a bucket the
    // largest over the chain (the workspace is sized for d_max chi, which bounds both)
    w.mmax = bkt ? bkt->mmax : s->mstruct;
    w.nmax = bkt ? bkt->nmax : s->nstruct;
    w.theta_stride = (size_t)w.mmax * w.nmax;
    w.theta64 = (s->prec == 0 || s->theta64) ? 1 : 0;
    w.theta = ws + s->lay.u_theta;
    w.gram = reinterpret_cast<double2*>(ws + s->lay.u_gram);
    w.refl = reinterpret_cast<double2*>(ws + s->lay.u_refl);
    w.tau = reinterpret_cast<double2*>(ws + s->lay.u_tau);
    w.dd = reinterpret_cast<double*>(ws + s->lay.u_dd);
    w.ee = reinterpret_cast<double*>(ws + s->lay.u_ee);
    w.logcap = s->logcap;
    w.logi = reinterpret_cast<int*>(ws + s->lay.u_logi);
    w.logcs = reinterpret_cast<double2*>(ws + s->lay.u_logcs);
    w.nrot = reinterpret_cast<int*>(ws + s->lay.u_nrot);
    w.sel = reinterpret_cast<int*>(ws + s->lay.u_sel);
    w.kout = reinterpret_cast<int*>(ws + s->lay.u_kout);
    w.sout = reinterpret_cast<double*>(ws + s->lay.u_sout);
    w.wout = reinterpret_cast<double*>(ws + s->lay.u_wout);
    w.V = reinterpret_cast<double2*>(ws + s->lay.u_V);
    w.zscratch = reinterpret_cast<double2*>(ws + s->lay.u_z);
    w.pscratch = reinterpret_cast<double2*>(ws + s->lay.u_p);
    w.flags = at<int>(s, s->lay.off_flags);
    w.counters = at<unsigned long long>(s, s->lay.off_flags + 8);
    w.gsz = reinterpret_cast<int*>(ws + s->lay.u_gsz);
    w.qra = reinterpret_cast<double2*>(ws + s->lay.u_qra);
    w.qtau = reinterpret_cast<double2*>(ws + s->lay.u_qtau);
    w.qr_route = s->prec == 0 ? 1 : 0;
    w.jacobi = s->prec == 0 ? 1 : 0;
    w.vld = s->prec == 0 ? w.nmax : s->chi;
    // Y = Theta~ V (m x r, r <= n) goes into the Gram slot, which is free once the Householder
    // reduction has read it; a bucket's items can have m > n, so its rows take max(m, n)
    w.Y = w.gram;
    w.ldy = std::max(w.mmax, w.nmax);
    w.ysz = (size_t)w.ldy * w.nmax;
    w.lsel = reinterpret_cast<double*>(ws + s->lay.u_lsel);
    // split mode with n <= 128 and chi <= 64 takes the bisection path (kernels in k_update.hip)
    w.fb = (s->prec == 1 && w.nmax <= 128 && s->chi <= 64) ? reinterpret_cast<int*>(ws + s->lay.u_fb) : nullptr;
    w.hvar = bkt ? bkt->hvar : s->hvar;
    return w;
}

static int run_layer(tn_state* s, int parity, int slot, const unsigned char* mask_dev) {
    const int nb = parity <= s->L - 2 ? ((s->L - 2 - parity) / 2 + 1) : 0;
    if (nb == 0) return TN_OK;
    DevState ds = dev_state(s);
    const long total = (long)s->B * nb;
    double* glog = at<double>(s, s->lay.off_glog);
    double* gwt = at<double>(s, s->lay.off_gwt);
    // Items of one layer are independent.  With two workspace slots, chunks run on the main
    // stream or on aux (with aux's own slot), forked after the work already on the main stream and
    // joined back before the layer's reduction.  (Ordering the heavy phases of the two streams
    // into one chain, so that light phases of one chunk run beside heavy phases of the other,
    // measured no faster than plain alternation: the kernels share the compute units' LDS
    // bandwidth.)
    // Buckets (bucketing 1) when the layer has at least one item per compute unit; a smaller layer
    // is latency-bound and goes out whole, since one launch sequence then beats several in a row.
    // Bucketing 2 buckets every layer.
    const bool bucketed = s->bucketing == 2 || (s->bucketing == 1 && total >= s->ncu);
    long nch = 0;
    if (bucketed)
        for (const tn_state::Bucket& bkt : s->bk[parity]) nch += ((long)s->B * bkt.count + s->chunk - 1) / s->chunk;
    else
        nch = (total + s->chunk - 1) / s->chunk;
    const bool two = s->nslots == 2 && s->overlap && s->aux && nch > 1;
    if (two) {
        HIPCHK(hipEventRecord(s->ev_fork, s->stream));
        HIPCHK(hipStreamWaitEvent(s->aux, s->ev_fork, 0));
    }
    // a bucket's items (or the layer's) go out in the fewest chunks of at most s->chunk, of equal
    // size; each chunk goes to the stream with less work queued so far, work counted as
    // items x order^3 (the Householder reduction's share)
    double load[2] = {0.0, 0.0};
    auto chunks = [&](long items, const tn_state::Bucket* bkt) -> int {
        const long nc = (items + s->chunk - 1) / s->chunk;
        const long per = (items + nc - 1) / nc;
        const double ord = bkt ? bkt->nmax : s->nstruct;
        for (long i0 = 0; i0 < items; i0 += per) {
            const int nitems = (int)std::min(per, items - i0);
            const int ws = two ? (load[1] < load[0] ? 1 : 0) : 0;
            load[ws] += (double)nitems * ord * ord * ord;
            DevWork w = chunk_work(s, parity, nb, slot, i0, nitems, mask_dev, ws, bkt);
            launch_layer_chunk(s->prec, ds, w, ws ? s->aux : s->stream, ws ? &s->prof2 : &s->prof, glog, gwt);
            HIPCHK(hipGetLastError());
        }
        return TN_OK;
    };
    if (bucketed) {
        for (const tn_state::Bucket& bkt : s->bk[parity]) {
            const int rc = chunks((long)s->B * bkt.count, &bkt);
            if (rc != TN_OK) return rc;
        }
    } else {
        const int rc = chunks(total, nullptr);
        if (rc != TN_OK) return rc;
    }
    if (two) {
        HIPCHK(hipEventRecord(s->ev_join, s->aux));
        HIPCHK(hipStreamWaitEvent(s->stream, s->ev_join, 0));
    }
    launch_reduce_items(ds, nb, parity, mask_dev, glog, gwt, s->stream);
    HIPCHK(hipGetLastError());
    return TN_OK;
}

// Sequential sweep (Sec. 2.3, eq. ShiftCenter): one bond of every unmasked instance per launch
// sequence, with the orthogonality centre on one of the bond's sites.  gate: the layer's gate
// in `slot`, or the identity (a centre shift); right: the centre leaves on site bond+1.
static int run_bond(tn_state* s, int bond, int slot, bool gate, bool right, const unsigned char* mask_dev) {
    DevState ds = dev_state(s);
    double* glog = at<double>(s, s->lay.off_glog);
    double* gwt = at<double>(s, s->lay.off_gwt);
    for (long i0 = 0; i0 < s->B; i0 += s->chunk) {
        const int nitems = (int)std::min((long)s->chunk, (long)s->B - i0);
        DevWork w = chunk_work(s, bond, 1, slot, i0, nitems, mask_dev);
        w.unitw = 1;
        w.rmove = right ? 1 : 0;
        w.skip_gate = gate ? 0 : 1;
        launch_layer_chunk(s->prec, ds, w, s->stream, &s->prof, glog, gwt);
        HIPCHK(hipGetLastError());
    }
    launch_reduce_items(ds, 1, bond, mask_dev, glog, gwt, s->stream);
    HIPCHK(hipGetLastError());
    return TN_OK;
}

// One Trotter step by the sweep.  Passes (the layers of the step, in order) alternate direction,
// the first going left to right; before each gate the centre is shifted one bond at a time
// until it sits on the bond; after the last pass it returns to site 0, so that between steps
// every tensor but the first is right-canonical (the storage form of the layer schedule).
static int sweep_step(tn_state* s, const std::vector<std::pair<int, int>>& layers, const unsigned char* mask_dev) {
    int c = 0, rc;
    bool right = true;
    for (auto& ly : layers) {
        std::vector<int> bonds;
        for (int b = ly.first; b <= s->L - 2; b += 2) bonds.push_back(b);
        if (!right) std::reverse(bonds.begin(), bonds.end());
        for (int b : bonds) {
            for (; c < b; ++c)
                if ((rc = run_bond(s, c, 0, false, true, mask_dev))) return rc;
            for (; c > b + 1; --c)
                if ((rc = run_bond(s, c - 1, 0, false, false, mask_dev))) return rc;
            if ((rc = run_bond(s, b, ly.second, true, right, mask_dev))) return rc;
            c = right ? b + 1 : b;
        }
        right = !right;
    }
    for (; c > 0; --c)
        if ((rc = run_bond(s, c - 1, 0, false, false, mask_dev))) return rc;
    return TN_OK;
}

static int run_step(tn_state* s, const std::vector<std::pair<int, int>>& layers, const unsigned char* mask_dev) {
    if (s->schedule == TN_SCHED_SWEEP) return sweep_step(s, layers, mask_dev);
    int rc;
    for (auto& ly : layers)
        if ((rc = run_layer(s, ly.first, ly.second, mask_dev))) return rc;
    return TN_OK;
}

// Autotuner: for n <= 128 two Householder kernels exist (MFMA block columns, wave tiles).  On the
// first Trotter step of a state both run on the Gram matrices of the state's own first chunk
// (Theta, gate and Gram are recomputed by the real step, the Householder kernels write only
// workspace), three times each, and the faster median is kept for the state's lifetime.
// A chunk too small to time against launch overhead keeps the default (MFMA) kernel, and the
// other kernel is taken only when it is clearly faster, so that the choice (and with it the
// rounding of the results) does not follow timing noise from run to run.
#define TUNE_MIN_ITEMS 2048
#define TUNE_MARGIN 0.95f
static int autotune(tn_state* s, int slot) {
    if (s->tuned) return TN_OK;
    s->tuned = 1;
    const int nb = (s->L - 2) / 2 + 1;  // parity 0 bonds
    // what is timed: the first chunk of each size class of the parity-0 buckets (the parity-1
    // buckets of a class take the same choice), or the first chunk of the layer when bucketing is
    // off; only orders <= 128 have two Householder variants
    std::vector<std::pair<int, const tn_state::Bucket*>> cand;
    if (s->bucketing) {
        for (const tn_state::Bucket& bkt : s->bk[0])
            if (bkt.nmax <= 128) cand.push_back({size_class(bkt.nmax), &bkt});
    } else if (s->nstruct <= 128) {
        cand.push_back({size_class(s->nstruct), nullptr});
    }
    int choice[4] = {-1, -1, -1, -1};
    float tms[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (!cand.empty()) {
        DevState ds = dev_state(s);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        for (const auto& c : cand) {
            const int cls = c.first;
            const long items = (long)s->B * (c.second ? c.second->count : nb);
            const int nitems = (int)std::min((long)s->chunk, items);
            if (nitems < TUNE_MIN_ITEMS || choice[cls] >= 0) continue;
            DevWork w = chunk_work(s, 0, nb, slot, 0, nitems, nullptr, 0, c.second);
            launch_update_prefix(s->prec, ds, w, s->stream);
            HIPCHK(hipGetLastError());
            for (int v = 0; v < 2; ++v) {
                float t[3];
                for (int rep = 0; rep < 3; ++rep) {
                    HIPCHK(hipEventRecord(e0, s->stream));
                    launch_hetrd_variant(ds, w, v, s->stream);
                    HIPCHK(hipEventRecord(e1, s->stream));
                    HIPCHK(hipEventSynchronize(e1));
                    HIPCHK(hipEventElapsedTime(&t[rep], e0, e1));
                }
                std::sort(t, t + 3);
                tms[cls][v] = t[1];
            }
            choice[cls] = tms[cls][1] < TUNE_MARGIN * tms[cls][0] ? 1 : 0;
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
    for (int p = 0; p < 2; ++p)
        for (tn_state::Bucket& bkt : s->bk[p]) {
            const int cls = size_class(bkt.nmax);
            if (choice[cls] >= 0) {
                bkt.hvar = choice[cls];
                bkt.tune_ms[0] = tms[cls][0];
                bkt.tune_ms[1] = tms[cls][1];
            }
        }
    // the state-wide variant (unbucketed layers, sweeps) is the choice of the largest class timed
    for (int cls = 3; cls >= 0; --cls)
        if (choice[cls] >= 0) {
            s->hvar = choice[cls];
            s->tune_ms[0] = tms[cls][0];
            s->tune_ms[1] = tms[cls][1];
            if (!s->bucketing)
                for (int p = 0; p < 2; ++p)
                    for (tn_state::Bucket& bkt : s->bk[p]) bkt.hvar = choice[cls];
            break;
        }
    return TN_OK;
}

extern "C" int tebd_step(void* h, double dt, int order, int n_steps, const unsigned char* mask,
                         double* trunc_weight_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (order != 1 && order != 2) return fail(TN_EINVAL, "order must be 1 or 2");
    if (n_steps < 0) return fail(TN_EINVAL, "n_steps must be >= 0");
    if (!(std::isfinite(dt))) return fail(TN_EINVAL, "dt must be finite");
    int rc;
    // layer sequence (parity, slot); slot 0 = dt (order 1) or dt/2 (order 2), slot 1 = dt (order 2)
    std::vector<std::pair<int, int>> layers;
    if (order == 1) {
        if ((rc = upload_gates(s, 0, dt))) return rc;
        layers = {{0, 0}, {1, 0}};
    } else {
        if ((rc = upload_gates(s, 0, dt / 2))) return rc;
        if ((rc = upload_gates(s, 1, dt))) return rc;
        layers = {{1, 0}, {0, 1}, {1, 0}};
    }
    if (!s->tuned && n_steps > 0 && (rc = autotune(s, 0))) return rc;
    const unsigned char* mdev = nullptr;
    if (mask) {
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_mask, mask, s->B, hipMemcpyHostToDevice, s->stream));
        mdev = reinterpret_cast<const unsigned char*>(s->arena + s->lay.off_mask);
    }
    // Untimed steps replay one captured graph of the step's layers per schedule, order and
    // masking (kernel launches only: no memset or copy nodes).  Gates and the mask live in fixed
    // arena slots that the copies above refill, so a new dt or mask needs no re-capture.  The
    // library's stream must be a created stream for capture.
    if (s->use_graph && !s->prof.on && s->stream != nullptr && n_steps > 0) {
        hipGraphExec_t& gx = s->gexec[s->schedule][order][mdev ? 1 : 0];
        if (!gx) {
            HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            const int crc = run_step(s, layers, mdev);
            hipGraph_t graph = nullptr;
            const hipError_t ce = hipStreamEndCapture(s->stream, &graph);
            if (crc) {
                if (graph) hipGraphDestroy(graph);
                return crc;
            }
            if (ce != hipSuccess) return fail(TN_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
            const hipError_t ie = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                gx = nullptr;
                return fail(TN_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            }
        }
        for (int st = 0; st < n_steps; ++st) HIPCHK(hipGraphLaunch(gx, s->stream));
    } else {
        for (int st = 0; st < n_steps; ++st)
            if ((rc = run_step(s, layers, mdev))) return rc;
    }
    if ((rc = check_flags(s))) {
        if (trunc_weight_out)
            hipMemcpy(trunc_weight_out, s->arena + s->lay.off_trunc, (size_t)s->B * 8, hipMemcpyDeviceToHost);
        return rc;
    }
    if (trunc_weight_out) {
        HIPCHK(hipMemcpyAsync(trunc_weight_out, s->arena + s->lay.off_trunc, (size_t)s->B * 8, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return TN_OK;
}

// ------------------------------------------------------------------ measurement
static MeasWork meas_work(const Layout& ly, tn_state* s, char* ws, double2* ceach, double* nrm, int b0, int nbm) {
    MeasWork mw;
    mw.b0 = b0;
    mw.nbm = nbm;
    mw.R = ws + ly.m_R;
    mw.E = ws + ly.m_E;
    mw.X = ws + ly.m_X;
    mw.Y = ws + ly.m_Y;
    mw.W = ws + ly.m_W;
    mw.C = ceach + (size_t)b0 * s->L * s->L;
    mw.nrm = nrm + b0;
    return mw;
}

// per instance: normalization or the lognorm scale; norm_out
__global__ void k_meas_scale(DevState s, double2* Ceach, double* nrm, int mode) {
    const int b = blockIdx.x;
    const int L = s.L;
    double f;
    double n = nrm[b];
    if (mode == 0) f = 1.0 / n;                          // normalized
    else if (mode == 1) f = exp(2.0 * s.lognorm[b]);      // linear (unnormalized)
    else f = 1.0 / n;                                     // MPDO: divide by trace
    for (int e = threadIdx.x; e < L * L; e += blockDim.x) Ceach[(size_t)b * L * L + e] = cscale(Ceach[(size_t)b * L * L + e], f);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (mode == 2) nrm[b] = n * exp(s.lognorm[b]);
        else nrm[b] = n * exp(2.0 * s.lognorm[b]);
    }
}
// batch mean and sample variance per entry (divisor B - 1, around the arithmetic mean; fixed
// summation order); with ratio the mean entry is sum_b C_b / sum_b <psi_b|psi_b> (the variance
// stays that of the per-instance values around their arithmetic mean)
__global__ void k_meas_stats(int B, int LL, const double2* Ceach, const double* nrm, int ratio, double2* mean,
                             double* var) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= LL) return;
    double2 m = mk(0, 0);
    for (int b = 0; b < B; ++b) m = cadd(m, Ceach[(size_t)b * LL + e]);
    double nsum = 0.0;
    if (ratio)
        for (int b = 0; b < B; ++b) nsum += nrm[b];
    const double2 csum = m;
    m = cscale(m, 1.0 / B);
    double v = 0.0;
    for (int b = 0; b < B; ++b) {
        double2 d = csub(Ceach[(size_t)b * LL + e], m);
        v += d.x * d.x + d.y * d.y;
    }
    mean[e] = ratio ? cscale(csum, 1.0 / nsum) : m;
    var[e] = B > 1 ? v / (B - 1) : 0.0;
}

// the measurement sweep of every instance of ds, with workspace ws, per-instance results ce
// and nr and batch statistics cmean, cvar, all launched on st
static int run_measure(tn_state* s, const DevState& ds, char* ws, double2* ce, double* nr, double2* cmean,
                       double* cvar, int normalize, hipStream_t st, const Layout* mly = nullptr, int group = 0) {
    const Layout& ly = mly ? *mly : s->lay;
    const int gsz = group > 0 ? group : s->nbm;
    for (int b0 = 0; b0 < s->B; b0 += gsz) {
        int nbm = std::min(gsz, s->B - b0);
        MeasWork mw = meas_work(ly, s, ws, ce, nr, b0, nbm);
        if (s->kind == TN_KIND_MPDO) launch_measure_mpdo(s->prec, ds, mw, st);
        else launch_measure_mps(s->prec, ds, mw, st);
        HIPCHK(hipGetLastError());
    }
    // normalize 0 and 2 on an MPS keep <psi|O|psi> per instance (linear QSD); 2 also divides the
    // batch sum by the summed norms
    const bool linear = s->kind == TN_KIND_MPS && (normalize == 0 || normalize == 2);
    const int ratio = s->kind == TN_KIND_MPS && normalize == 2;
    int mode = s->kind == TN_KIND_MPDO ? 2 : (linear ? 1 : 0);
    hipLaunchKernelGGL(k_meas_scale, dim3(s->B), dim3(256), 0, st, ds, ce, nr, mode);
    const int LL = s->L * s->L;
    hipLaunchKernelGGL(k_meas_stats, dim3((LL + 255) / 256), dim3(256), 0, st, s->B, LL, ce, nr, ratio, cmean, cvar);
    HIPCHK(hipGetLastError());
    return TN_OK;
}

static int copy_measure_out(tn_state* s, const double2* ce, const double* nr, const double2* cmean, const double* cvar,
                            double* C_mean, double* C_var, double* C_each, double* norm_out, hipStream_t st) {
    const int LL = s->L * s->L;
    HIPCHK(hipMemcpyAsync(C_mean, cmean, (size_t)LL * 16, hipMemcpyDeviceToHost, st));
    if (C_var) HIPCHK(hipMemcpyAsync(C_var, cvar, (size_t)LL * 8, hipMemcpyDeviceToHost, st));
    if (C_each) HIPCHK(hipMemcpyAsync(C_each, ce, (size_t)s->B * LL * 16, hipMemcpyDeviceToHost, st));
    if (norm_out) HIPCHK(hipMemcpyAsync(norm_out, nr, (size_t)s->B * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return TN_OK;
}

extern "C" int measure_corr(void* h, int normalize, double* C_mean, double* C_var, double* C_each, double* norm_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (!C_mean) return fail(TN_EINVAL, "C_mean is null");
    DevState ds = dev_state(s);
    double2* ce = at<double2>(s, s->lay.off_ceach);
    double* nr = at<double>(s, s->lay.off_nrm);
    double2* cm = at<double2>(s, s->lay.off_cmean);
    double* cv = at<double>(s, s->lay.off_cvar);
    prof_begin(&s->prof, TN_K_MEASURE, s->stream);
    int rc = run_measure(s, ds, s->arena + s->lay.off_ws, ce, nr, cm, cv, normalize, s->stream);
    if (rc != TN_OK) return rc;
    prof_end(&s->prof, TN_K_MEASURE, s->stream);
    return copy_measure_out(s, ce, nr, cm, cv, C_mean, C_var, C_each, norm_out, s->stream);
}

extern "C" int measure_corr_noalloc(void* h, int normalize, double* C_mean, double* C_var, double* C_each,
                                    double* norm_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (!C_mean) return fail(TN_EINVAL, "C_mean is null");
    if (!s->scratch) return fail(TN_EHIP, "the static scratch of this state's device was not set up");
    // the largest group of instances whose workspace fits the scratch (at most the arena path's)
    Layout ml = s->lay;
    const size_t one = meas_sublayout(ml, s->L, s->chi, s->dmax, s->esz, 1);
    if (one > TN_SCRATCH_BYTES) {
        char buf[192];
        snprintf(buf, sizeof buf,
                 "measure_corr_noalloc: one instance needs %zu bytes of measurement workspace, above the "
                 "static scratch of %zu bytes (TN_SCRATCH_BYTES)", one, (size_t)TN_SCRATCH_BYTES);
        return fail(TN_ENOMEM, buf);
    }
    int group = (int)std::min<size_t>((size_t)std::min(s->nbm, s->B), TN_SCRATCH_BYTES / one);
    while (group > 1 && meas_sublayout(ml, s->L, s->chi, s->dmax, s->esz, group) > TN_SCRATCH_BYTES) --group;
    meas_sublayout(ml, s->L, s->chi, s->dmax, s->esz, group);
    DevState ds = dev_state(s);
    double2* ce = at<double2>(s, s->lay.off_ceach);
    double* nr = at<double>(s, s->lay.off_nrm);
    double2* cm = at<double2>(s, s->lay.off_cmean);
    double* cv = at<double>(s, s->lay.off_cvar);
    int rc = run_measure(s, ds, s->scratch, ce, nr, cm, cv, normalize, s->stream, &ml, group);
    if (rc != TN_OK) return rc;
    return copy_measure_out(s, ce, nr, cm, cv, C_mean, C_var, C_each, norm_out, s->stream);
}

// ------------------------------------------------------------------ asynchronous measurement
// offsets inside the second buffer: the snapshot repeats the arena's [off_tens, off_trunc)
// range byte for byte, so its pointers keep the arena's relative offsets
struct AsyncLayout {
    size_t snap, nrm, ceach, cmean, cvar, ws, total;
};
static AsyncLayout async_layout(const tn_state* s) {
    AsyncLayout a;
    size_t o = 0;
    a.snap = o; o = al(o + (s->lay.off_trunc - s->lay.off_tens));
    a.nrm = o; o = al(o + (size_t)s->B * 8);
    a.ceach = o; o = al(o + (size_t)s->B * s->L * s->L * 16);
    a.cmean = o; o = al(o + (size_t)s->L * s->L * 16);
    a.cvar = o; o = al(o + (size_t)s->L * s->L * 8);
    a.ws = o; o = al(o + s->lay.m_bytes);
    a.total = o;
    return a;
}

extern "C" size_t tn_measure_async_bytes(const void* h) {
    const tn_state* s = reinterpret_cast<const tn_state*>(h);
    return s ? async_layout(s).total : 0;
}

extern "C" int tn_measure_async_enable(void* h, void* buf, size_t bytes) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (!buf) return fail(TN_EINVAL, "buffer is null");
    if (reinterpret_cast<uintptr_t>(buf) % 256 != 0) return fail(TN_EINVAL, "buffer is not 256-byte aligned");
    if (s->apending) return fail(TN_EINVAL, "a measurement is outstanding");
    const AsyncLayout a = async_layout(s);
    if (bytes < a.total) return fail(TN_ENOMEM, "buffer smaller than tn_measure_async_bytes");
    if (!s->mstream) HIPCHK(hipStreamCreateWithFlags(&s->mstream, hipStreamNonBlocking));
    if (!s->ev_snap) HIPCHK(hipEventCreateWithFlags(&s->ev_snap, hipEventDisableTiming));
    s->abuf = reinterpret_cast<char*>(buf);
    s->a_snap = a.snap;
    s->a_nrm = a.nrm;
    s->a_ceach = a.ceach;
    s->a_cmean = a.cmean;
    s->a_cvar = a.cvar;
    s->a_ws = a.ws;
    s->a_total = a.total;
    return TN_OK;
}

extern "C" int measure_corr_start(void* h, int normalize) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (!s->abuf) return fail(TN_EINVAL, "asynchronous measurement not enabled (tn_measure_async_enable)");
    if (s->apending) return fail(TN_EINVAL, "a measurement is outstanding (measure_corr_finish)");
    // snapshot in the order of the work already queued on the state's stream
    char* snap = s->abuf + s->a_snap;
    HIPCHK(hipMemcpyAsync(snap, s->arena + s->lay.off_tens, s->lay.off_trunc - s->lay.off_tens,
                          hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipEventRecord(s->ev_snap, s->stream));
    HIPCHK(hipStreamWaitEvent(s->mstream, s->ev_snap, 0));
    DevState ds = dev_state(s);
    ds.tens = snap;
    ds.lam = reinterpret_cast<double*>(snap + (s->lay.off_lam - s->lay.off_tens));
    ds.dims = reinterpret_cast<int*>(snap + (s->lay.off_dims - s->lay.off_tens));
    ds.lognorm = reinterpret_cast<double*>(snap + (s->lay.off_lognorm - s->lay.off_tens));
    ds.trunc = nullptr;
    prof_begin(&s->prof3, TN_K_MEASURE, s->mstream);
    int rc = run_measure(s, ds, s->abuf + s->a_ws, reinterpret_cast<double2*>(s->abuf + s->a_ceach),
                         reinterpret_cast<double*>(s->abuf + s->a_nrm), reinterpret_cast<double2*>(s->abuf + s->a_cmean),
                         reinterpret_cast<double*>(s->abuf + s->a_cvar), normalize, s->mstream);
    if (rc != TN_OK) return rc;
    prof_end(&s->prof3, TN_K_MEASURE, s->mstream);
    s->apending = true;
    return TN_OK;
}

extern "C" int measure_corr_finish(void* h, double* C_mean, double* C_var, double* C_each, double* norm_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (!s->apending) return fail(TN_EINVAL, "no measurement outstanding (measure_corr_start)");
    if (!C_mean) return fail(TN_EINVAL, "C_mean is null");
    s->apending = false;
    return copy_measure_out(s, reinterpret_cast<double2*>(s->abuf + s->a_ceach),
                            reinterpret_cast<double*>(s->abuf + s->a_nrm), reinterpret_cast<double2*>(s->abuf + s->a_cmean),
                            reinterpret_cast<double*>(s->abuf + s->a_cvar), C_mean, C_var, C_each, norm_out, s->mstream);
}

// ------------------------------------------------------------------ dissipative step
extern "C" int apply_jumps(void* h, int mode, double dt, const double* rnd, int noise_kind, int* jumped_out,
                           unsigned char* mask_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (s->njump == 0) return fail(TN_EINVAL, "model has no jump operators");
    DevState ds = dev_state(s);
    const int* jsite = at<int>(s, s->lay.off_jsite);
    const double2* jop = at<double2>(s, s->lay.off_jop);
    const double* gam = at<double>(s, s->lay.off_gam);
    const bool qt = mode == TN_MODE_QT || mode == TN_MODE_QT_SHIFT;
    const bool qsd = mode == TN_MODE_QSD || mode == TN_MODE_QSD_SHIFT;
    const bool shifted = mode == TN_MODE_QT_SHIFT || mode == TN_MODE_QSD_SHIFT;
    if (!qt && !qsd && mode != TN_MODE_KRAUS) return fail(TN_EINVAL, "unknown mode");
    if (qt && s->kind != TN_KIND_MPS) return fail(TN_EINVAL, "QT jumps need kind MPS");
    if (qsd && s->kind != TN_KIND_MPS) return fail(TN_EINVAL, "QSD noise needs kind MPS");
    if ((qt || qsd) && !rnd) return fail(TN_EINVAL, "rnd is null");
    if (qsd && noise_kind != 0 && noise_kind != 1) return fail(TN_EINVAL, "unknown noise kind");
    if (mode == TN_MODE_KRAUS && s->kind != TN_KIND_PURIFIED)
        return fail(TN_EINVAL, "Kraus compression needs kind PURIFIED");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(TN_EINVAL, "dt must be finite and >= 0");
    if (qt || qsd) {
        // uniforms (QT draws, binary increments) in [0, 1]; Gaussian increments finite
        const bool unif = qt || noise_kind == 1;
        const size_t n = qt ? (size_t)s->B : (size_t)s->B * s->njump * (noise_kind == 0 ? 2 : 1);
        for (size_t e = 0; e < n; ++e)
            if (!std::isfinite(rnd[e]) || (unif && !(rnd[e] >= 0.0 && rnd[e] <= 1.0)))
                return fail(TN_EINVAL, unif ? "rnd must hold uniforms in [0, 1]" : "rnd must be finite");
    }
    prof_begin(&s->prof, TN_K_JUMPS, s->stream);
    // host copies of L (row-major 2x2 per channel) and L^+L for the closing kernels
    std::vector<double2> jl(4 * s->njump), jL(4 * s->njump);
    for (int q = 0; q < s->njump; ++q) {
        double2 o[4];
        for (int e = 0; e < 4; ++e) o[e] = mk(s->model.jump_op[8 * q + 2 * e], s->model.jump_op[8 * q + 2 * e + 1]);
        for (int e = 0; e < 4; ++e) jL[4 * q + e] = o[e];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                double2 acc = mk(0, 0);
                for (int k = 0; k < 2; ++k) cfmac(acc, o[k * 2 + r], o[k * 2 + c]);
                jl[4 * q + r * 2 + c] = acc;
            }
    }
    double* vals = at<double>(s, s->lay.off_vals);
    double2* lvals = shifted ? at<double2>(s, s->lay.off_lval) : nullptr;
    if (qt) {
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_rnd, rnd, (size_t)s->B * 8, hipMemcpyHostToDevice, s->stream));
        for (int b0 = 0; b0 < s->B; b0 += s->nbm) {
            int nbm = std::min(s->nbm, s->B - b0);
            MeasWork mw = meas_work(s->lay, s, s->arena + s->lay.off_ws, at<double2>(s, s->lay.off_ceach), at<double>(s, s->lay.off_nrm), b0, nbm);
            launch_jump_expect(s->prec, ds, mw, s->njump, s->model.jump_site.data(), jl.data(), vals,
                               shifted ? jL.data() : nullptr, lvals, s->stream);
            launch_qt_apply(s->prec, ds, b0, nbm, dt, s->njump, jsite, jop, gam, vals, lvals, mw.nrm,
                            at<double>(s, s->lay.off_rnd), at<int>(s, s->lay.off_jumped),
                            reinterpret_cast<unsigned char*>(s->arena + s->lay.off_mask), s->stream);
            HIPCHK(hipGetLastError());
        }
        if (jumped_out)
            HIPCHK(hipMemcpyAsync(jumped_out, s->arena + s->lay.off_jumped, (size_t)s->B * 4, hipMemcpyDeviceToHost,
                                  s->stream));
        if (mask_out)
            HIPCHK(hipMemcpyAsync(mask_out, s->arena + s->lay.off_mask, (size_t)s->B, hipMemcpyDeviceToHost, s->stream));
    } else if (qsd) {
        size_t n = (size_t)s->B * s->njump * (noise_kind == 0 ? 2 : 1);
        HIPCHK(hipMemcpyAsync(s->arena + s->lay.off_rnd, rnd, n * 8, hipMemcpyHostToDevice, s->stream));
        if (!shifted) {
            launch_qsd_apply(s->prec, ds, 0, s->B, dt, s->njump, jsite, jop, gam, at<double>(s, s->lay.off_rnd),
                             noise_kind, nullptr, nullptr, s->stream);
        } else {
            for (int b0 = 0; b0 < s->B; b0 += s->nbm) {
                int nbm = std::min(s->nbm, s->B - b0);
                MeasWork mw = meas_work(s->lay, s, s->arena + s->lay.off_ws, at<double2>(s, s->lay.off_ceach), at<double>(s, s->lay.off_nrm), b0, nbm);
                launch_jump_expect(s->prec, ds, mw, s->njump, s->model.jump_site.data(), jl.data(), vals, jL.data(),
                                   lvals, s->stream);
                launch_qsd_apply(s->prec, ds, b0, nbm, dt, s->njump, jsite, jop, gam,
                                 at<double>(s, s->lay.off_rnd), noise_kind, lvals, mw.nrm, s->stream);
            }
        }
        HIPCHK(hipGetLastError());
    } else if (mode == TN_MODE_KRAUS) {
        std::vector<double2> hop(4 * s->njump);
        for (int q = 0; q < 4 * s->njump; ++q) hop[q] = mk(s->model.jump_op[2 * q], s->model.jump_op[2 * q + 1]);
        launch_kraus(s->prec, ds, dt, s->njump, s->model.jump_site.data(), hop.data(), s->model.gamma.data(), s->chik,
                     s->stream);
        HIPCHK(hipGetLastError());
    } else {
        return fail(TN_EINVAL, "unknown mode");
    }
    prof_end(&s->prof, TN_K_JUMPS, s->stream);
    HIPCHK(hipStreamSynchronize(s->stream));
    return TN_OK;
}

// ------------------------------------------------------------------ autotuner report / override
extern "C" int tn_tuning(void* h, int set_variant, int* variant_out, float* ms_out) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    if (set_variant < -1 || set_variant > 1) return fail(TN_EINVAL, "variant must be -1, 0 or 1");
    if (set_variant >= 0) {
        hipStreamSynchronize(s->stream);
        s->hvar = set_variant;
        for (int p = 0; p < 2; ++p)
            for (tn_state::Bucket& bkt : s->bk[p]) bkt.hvar = set_variant;
        s->tuned = 1;
        drop_graphs(s);  // captured launches carry the old variant
    }
    if (variant_out) *variant_out = s->hvar;
    if (ms_out) {
        ms_out[0] = s->tune_ms[0];
        ms_out[1] = s->tune_ms[1];
    }
    return TN_OK;
}

// ------------------------------------------------------------------ graph replay switch
extern "C" int tn_graph_enable(void* h, int on) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    hipStreamSynchronize(s->stream);
    s->use_graph = on != 0;
    if (!s->use_graph) drop_graphs(s);
    return TN_OK;
}

extern "C" int tn_overlap(void* h, int on) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->overlap = on != 0;
    drop_graphs(s);  // captured steps carry the old stream pattern
    return TN_OK;
}

extern "C" int tn_theta_precision(void* h, int bits) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (bits != 32 && bits != 64) return fail(TN_EINVAL, "bits must be 32 or 64");
    if (s->prec == 0 && bits == 32) return fail(TN_EINVAL, "FP64 mode contracts in FP64 only");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->theta64 = bits == 64 ? 1 : 0;
    drop_graphs(s);  // captured steps carry the old kernels
    return TN_OK;
}

extern "C" int tn_buckets(void* h, int on, int parity, int* count, int* nmax, int* nbonds, int* hvar) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (on < -1 || on > 2 || parity < 0 || parity > 1) return fail(TN_EINVAL, "on must be -1, 0, 1 or 2, parity 0 or 1");
    if (on >= 0) {
        HIPCHK(hipStreamSynchronize(s->stream));
        s->bucketing = on;
        drop_graphs(s);  // captured steps carry the old chunking
    }
    const std::vector<tn_state::Bucket>& bk = s->bk[parity];
    if (count) *count = (int)bk.size();
    for (size_t i = 0; i < bk.size() && i < 4; ++i) {
        if (nmax) nmax[i] = bk[i].nmax;
        if (nbonds) nbonds[i] = bk[i].count;
        if (hvar) hvar[i] = bk[i].hvar;
    }
    return TN_OK;
}

extern "C" int tn_schedule(void* h, int schedule) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    if (schedule != TN_SCHED_LAYER && schedule != TN_SCHED_SWEEP) return fail(TN_EINVAL, "unknown schedule");
    HIPCHK(hipStreamSynchronize(s->stream));
    s->schedule = schedule;
    return TN_OK;
}

// ------------------------------------------------------------------ timing
extern "C" int tn_stats(void* h, int reset, long long* ql_fallback_items, long long* reorthogonalized_items) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    g_err.clear();
    if (!s) return fail(TN_EINVAL, "null handle");
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, s->arena + s->lay.off_flags + 8, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (ql_fallback_items) *ql_fallback_items = (long long)c[0];
    if (reorthogonalized_items) *reorthogonalized_items = (long long)c[1];
    if (reset) {
        HIPCHK(hipMemsetAsync(s->arena + s->lay.off_flags + 8, 0, sizeof c, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return TN_OK;
}

extern "C" int tn_prof_enable(void* h, int on) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    hipStreamSynchronize(s->stream);
    if (s->mstream) hipStreamSynchronize(s->mstream);
    for (Prof* p : {&s->prof, &s->prof2, &s->prof3}) {
        for (int k = 0; k < TN_K_COUNT; ++k) {
            for (auto& pr : p->ev[k]) {
                hipEventDestroy(pr.first);
                hipEventDestroy(pr.second);
            }
            p->ev[k].clear();
            p->open[k] = nullptr;
        }
        p->on = on != 0;
    }
    if (s->prof.ref) {
        hipEventDestroy(s->prof.ref);
        s->prof.ref = nullptr;
    }
    if (on) {
        HIPCHK(hipEventCreate(&s->prof.ref));
        HIPCHK(hipEventRecord(s->prof.ref, s->stream));
    }
    return TN_OK;
}

// Wall time during which at least one launch of the bucket was running (union of the launch
// intervals of both streams, measured from the common reference event).
extern "C" int tn_prof_busy(void* h, int kernel_id, double* busy_ms) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    if (kernel_id < 0 || kernel_id >= TN_K_COUNT) return fail(TN_EINVAL, "bad kernel id");
    if (!busy_ms) return fail(TN_EINVAL, "busy_ms is null");
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->mstream) HIPCHK(hipStreamSynchronize(s->mstream));
    *busy_ms = 0.0;
    if (!s->prof.ref) return TN_OK;
    std::vector<std::pair<double, double>> iv;
    for (Prof* p : {&s->prof, &s->prof2, &s->prof3})
        for (auto& pr : p->ev[kernel_id]) {
            float a = 0.0f, b = 0.0f;
            HIPCHK(hipEventElapsedTime(&a, s->prof.ref, pr.first));
            HIPCHK(hipEventElapsedTime(&b, s->prof.ref, pr.second));
            iv.push_back(std::make_pair((double)a, (double)b));
        }
    std::sort(iv.begin(), iv.end());
    double tot = 0.0, lo = 0.0, hi = -1.0;
    for (auto& x : iv) {
        if (x.first > hi) {
            if (hi > lo) tot += hi - lo;
            lo = x.first;
            hi = x.second;
        } else if (x.second > hi) {
            hi = x.second;
        }
    }
    if (hi > lo) tot += hi - lo;
    *busy_ms = tot;
    return TN_OK;
}

extern "C" int tn_prof_query(void* h, int kernel_id, double* total_ms, long long* launches) {
    tn_state* s = reinterpret_cast<tn_state*>(h);
    if (!s) return fail(TN_EINVAL, "null handle");
    if (kernel_id < 0 || kernel_id >= TN_K_COUNT) return fail(TN_EINVAL, "bad kernel id");
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->mstream) HIPCHK(hipStreamSynchronize(s->mstream));
    double tot = 0.0;
    long long cnt = 0;
    for (Prof* p : {&s->prof, &s->prof2, &s->prof3}) {
        for (auto& pr : p->ev[kernel_id]) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            tot += ms;
        }
        cnt += (long long)p->ev[kernel_id].size();
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return TN_OK;
}
