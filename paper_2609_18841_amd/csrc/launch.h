// Host-side declarations shared by the kernel files and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <vector>
#include "common.h"

#define TN_K_THETA   0
#define TN_K_GRAM    1
#define TN_K_HETRD   2
#define TN_K_STEQR   3
#define TN_K_VECS    4
#define TN_K_SPLIT   5
#define TN_K_MEASURE 6
#define TN_K_JUMPS   7
#define TN_K_COUNT   8

// Per-kernel event timing on the library stream.
struct Prof {
    bool on = false;
    hipEvent_t ref = nullptr;  // recorded when timing starts: common origin for both streams
    hipEvent_t open[TN_K_COUNT] = {};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[TN_K_COUNT];
};
void prof_begin(Prof* p, int id, hipStream_t st);
void prof_end(Prof* p, int id, hipStream_t st);

// update pipeline (k_update.hip)
void launch_layer_chunk(int prec, const DevState& s, const DevWork& w, hipStream_t st, Prof* prof,
                        double* glog, double* gwt);
// the same chunk in five phases (0 light, 1 heavy, 2 light, 3 heavy, 4 light); running phases 0..4
// in order equals launch_layer_chunk
void launch_layer_phase(int prec, const DevState& s, const DevWork& w, int phase, hipStream_t st, Prof* prof,
                        double* glog, double* gwt);
void launch_reduce_items(const DevState& s, int nb, int parity, const unsigned char* mask, const double* glog,
                         const double* gwt, hipStream_t st);
// pieces of the pipeline used by the autotuner: Theta, gate and Gram of a chunk (pure functions
// of the state), and one Householder variant on that Gram (workspace only)
void launch_update_prefix(int prec, const DevState& s, const DevWork& w, hipStream_t st);
void launch_hetrd_variant(const DevState& s, const DevWork& w, int variant, hipStream_t st);

// measurement workspace for a chunk of instances (k_measure.hip)
struct MeasWork {
    int b0, nbm;        // first instance, instances in this chunk
    void* R;            // (L+1) * nbm * chi*chi   right environments (T)
    void* E;            // nbm * chi*chi            running left environment (T)
    void* X;            // nbm * L * chi*chi        open strings (T)
    void* Y;            // nbm * L * chi*dmax*chi   X . B_j (T)
    void* W;            // nbm * chi*dmax*chi       conj(B_j) R_{j+1} (T)
    double2* C;         // nbm * L * L              correlation matrix per instance
    double* nrm;        // nbm                      <B|B> of the stored tensors
};
void launch_measure_mps(int prec, const DevState& s, const MeasWork& mw, hipStream_t st);
void launch_measure_mpdo(int prec, const DevState& s, const MeasWork& mw, hipStream_t st);
// right/left norm environments only (QT rates): fills mw.R for all sites and returns per-instance
// closings of the jump operators L^+L into vals[nbm * njump] (real parts) and, when jL is non-null,
// of L itself into lvals[nbm * njump] (complex); jLdL, jL: host arrays, njump*4 row-major 2x2
void launch_jump_expect(int prec, const DevState& s, const MeasWork& mw, int njump, const int* jsite,
                        const double2* jLdL, double* vals, const double2* jL, double2* lvals, hipStream_t st);

// dissipative kernels (k_jumps.hip); lvals == null: unshifted operators
void launch_qt_apply(int prec, const DevState& s, int b0, int nbm, double dt, int njump, const int* jsite,
                     const double2* jop, const double* gam, const double* vals, const double2* lvals,
                     const double* nrm, const double* rnd, int* jumped, unsigned char* mask, hipStream_t st);
void launch_qsd_apply(int prec, const DevState& s, int b0, int nbm, double dt, int njump, const int* jsite,
                      const double2* jop, const double* gam, const double* rnd, int noise_kind, const double2* lvals,
                      const double* nrm, hipStream_t st);
// jsite, jop, gam: host arrays (passed to the kernel by value)
void launch_kraus(int prec, const DevState& s, double dt, int njump, const int* jsite, const double2* jop,
                  const double* gam, int chik, hipStream_t st);
