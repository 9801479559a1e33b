/*
 * tebd.h -- C ABI of the MI355X (gfx950) batched TEBD-Lindblad hot path.
 *
 * Method: C. Chatelain, "A first introduction to Matrix Product State
 * algorithms for the integration of Lindblad equation".  The library evolves
 * a batch of B independent instances of one of three tensor-network forms of
 * an open chain of L sites:
 *   TN_KIND_MPS       pure states (quantum trajectories, Sec. 4.1; quantum state
 *                     diffusion, Sec. 4.2; unitary TEBD, Sec. 2.3), local dim 2;
 *   TN_KIND_MPDO      vectorized density matrix, local index m = n*2 + n'
 *                     (Sec. 3.1, eq. Choi / eq. MPDO), local dim 4;
 *   TN_KIND_PURIFIED  locally purified rho = X X^+ (Sec. 3.2, eq. Purified1), local
 *                     index p = n*chi_k + k; Kraus index only on jump sites.
 * Every instance is stored in Hastings form: psi = exp(lognorm) B_0 ... B_{L-1}
 * with site tensors B_i[a][p][c] (row-major, compact chi_l x d_i x chi_r) and
 * FP64 bond weights Lambda_b (bond b joins sites b and b+1, 0-based).
 *
 * Conventions shared by all entry points
 *   - Complex numbers cross the boundary as interleaved (re, im) doubles.
 *   - Host pointers are borrowed for the duration of the call and never retained.
 *   - The device arena is owned by the caller (e.g. a torch uint8 tensor); the
 *     library sub-allocates it and never frees it.  It must stay alive and
 *     unmoved until mps_free.
 *   - All device work is ordered on the HIP stream given to mps_alloc.  Entry
 *     points that return host outputs synchronize that stream before returning.
 *   - Return value 0 on success or a negative TN_E* code; mps_last_error()
 *     returns a thread-local message describing the last failure.
 *   - A handle must not be used by two host threads at once.
 */
#ifndef TEBD_H
#define TEBD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TN_OK        0
#define TN_EINVAL   -1   /* null pointer, bad size or shape, unsupported option */
#define TN_ENOMEM   -2   /* arena too small */
#define TN_EHIP     -3   /* a HIP runtime call failed */
#define TN_ENOCONV  -4   /* an eigensolver did not converge; results are still written */
#define TN_ENUMERIC -5   /* NaN/Inf detected in a result */

#define TN_KIND_MPS      0
#define TN_KIND_MPDO     1
#define TN_KIND_PURIFIED 2

#define TN_FP64  0   /* all contractions and storage in complex128 */
#define TN_SPLIT 1   /* complex64 storage of the site tensors; Theta and the measurement
                        sweep on the FP32 matrix cores (FP32 sums per 8-deep k-chunk, added in
                        FP64); Theta~, Gram, eigensolver, split, weights, norms and log-norms in
                        FP64 */

#define TN_MODE_QT    0  /* quantum-trajectory jumps, Sec. 4.1 */
#define TN_MODE_QSD   1  /* quantum-state-diffusion noise, Sec. 4.2 */
#define TN_MODE_KRAUS 2  /* Kraus-index compression of the purified form, Sec. 3.2 */
#define TN_MODE_QT_SHIFT  3  /* QT with shifted jump operators L_k - <L_k>, Sec. 4.1 */
#define TN_MODE_QSD_SHIFT 4  /* QSD with A_k = sqrt(gamma_k)(L_k - <L_k>) and the matching B, Sec. 4.2 */

#define TN_SCHED_LAYER 0  /* layer-parallel Hastings form: all bonds of a parity at once */
#define TN_SCHED_SWEEP 1  /* the paper's sequential sweep with the orthogonality centre, Sec. 2.3 */

#define TN_NOISE_GAUSS  0  /* dW = sqrt(dt) (x + i y)/sqrt(2), x, y ~ N(0,1) */
#define TN_NOISE_BINARY 1  /* dW = eta sqrt(dt), eta = -1 if u < 1/2 else +1 (the paper's choice) */

#define TN_MAX_JUMPS 256  /* jump channels per model */

/* Model of Sec. 2.1: H = sum_b h_b with two-site terms h_b on sites (b, b+1),
 * and local jump operators L_k on site jump_site[k] with rate gamma[k]
 * (Sec. 1 eq. Lindblad; eq. LindbladLocal for how their -i/2 gamma L^+L parts are
 * shared between bonds). */
typedef struct tn_model {
    int L;                    /* number of sites, >= 2 */
    int d;                    /* local Hilbert dimension; must be 2 */
    const double* h_bond;     /* (L-1) * 16 complex: 4x4 [out, in] in the basis n_b*2 + n_{b+1} */
    int n_jumps;              /* 0 .. TN_MAX_JUMPS (e.g. dephasing on every site plus drives) */
    const int* jump_site;     /* n_jumps sites, 0-based */
    const double* jump_op;    /* n_jumps * 4 complex: 2x2 [out, in] local operator (no string) */
    const double* gamma;      /* n_jumps rates >= 0 */
} tn_model;
/* mps_alloc refuses (TN_EINVAL) a model whose h_bond, jump_op or gamma holds a value that is not
 * finite. */

/* Bytes of device arena needed for a state of the given shape plus the
 * workspace of one chunk of chunk_items two-site updates (chunk_items <= 0:
 * the library's default).  Returns 0 on invalid arguments. */
size_t mps_arena_bytes(int kind, int L, int batch, int chi_max, int chi_k_max,
                       int precision, int chunk_items);

/* Create `batch` instances of the product state init_occ (L ints in {0,1}); all
 * bond dimensions 1.  MPDO: rho = |occ><occ|.  PURIFIED: X = |occ> with a Kraus
 * index of dimension chi_k_max on every jump site (unused columns zero).
 * chi_max in 1..256 caps every bond dimension.  With D_b the largest bond dimensions the chain
 * allows under chi_max, every bond's eigenproblem must stay of order <= 512 (split: the Gram
 * order d_{b+1} D_{b+2}; FP64: min of the two sides of Theta, wide Theta taking the QR route) and
 * Theta's sides <= 1024; TN_EINVAL otherwise (e.g. MPDO, FP64, L = 8, chi = 256 is accepted: its
 * Theta reaches 64 x 1024 but its eigenproblems 256).  sv_cutoff: singular values
 * sigma_a <= sv_cutoff * sigma_0 are discarded (Sec. 2.2 truncation).
 * arena: device pointer, arena_bytes >= mps_arena_bytes(...).  hip_stream: a
 * hipStream_t (NULL = default stream).  On success *out is a new handle. */
int mps_alloc(void** out, int kind, const tn_model* model, int batch, int chi_max,
              int chi_k_max, int precision, const int* init_occ, double sv_cutoff,
              void* arena, size_t arena_bytes, void* hip_stream);

/* Apply n_steps Trotter steps of size dt (Sec. 2.3; order 1: odd bonds then
 * even bonds; order 2: even dt/2, odd dt, even dt/2; bonds named by their
 * 1-based left site).  Gates are built in FP64 on the host: exp(-i h^eff_b tau)
 * for MPS and PURIFIED (h^eff: eq. EffHamiltonian shared per eq. LindbladLocal;
 * identity on Kraus indices), exp(l_b tau) for MPDO (eq. Liouvillian, row-major
 * vectorization).  Each two-site update forms Theta (eq. Theta / ThetaPurified),
 * splits it by a truncated FP64 SVD and stores it back in Hastings form; the
 * discarded weight (eq. HilbertSchmidtNorm) is accumulated per instance.
 * mask: B bytes or NULL; instances with mask[b] != 0 are not evolved.
 * trunc_weight_out: B doubles or NULL, receives the accumulated discarded weight. */
int tebd_step(void* s, double dt, int order, int n_steps, const unsigned char* mask,
              double* trunc_weight_out);

/* Dissipative part of one time step, on every instance.
 * TN_MODE_QT (MPS): rates p_k = gamma_k dt <L_k^+L_k>/<psi|psi> (eq. TransitionRate);
 *   rnd = B uniforms; jump k where sum_{k'<k} p_k' <= u < sum_{k'<=k} p_k'; the jumped
 *   state is L_k psi.  lognorm is reset so that the state is normalized.
 *   jumped_out[b] = k or -1, mask_out[b] = (k >= 0) (both B, may be NULL).
 * TN_MODE_QSD (MPS): psi <- prod_k (1 + dW_k sqrt(gamma_k) L_k) psi (Sec. 4.2), no
 *   renormalization.  rnd = B*n_jumps*2 normals (GAUSS) or B*n_jumps uniforms (BINARY).
 * TN_MODE_KRAUS (PURIFIED): on each jump site, rho -> rho + gamma dt L rho L^+ then the
 *   Kraus index is compressed back to chi_k_max (eq. MatrixR, eq. NewPurified); rnd NULL.
 * Shifted modes, with l_k = <psi|L_k|psi>/<psi|psi> of the state on entry (every l_k of a call
 * is taken before any of its factors is applied):
 * TN_MODE_QT_SHIFT (MPS): as TN_MODE_QT with Delta_k = -l_k: rates gamma_k dt (<L_k^+L_k> -
 *   |l_k|^2), the jumped state is (L_k - l_k) psi; without a jump each channel's factor
 *   1 + dt gamma_k (conj(l_k) L_k - |l_k|^2/2), the state-dependent single-site part of the
 *   shifted h^eff to first order, is applied in channel order (the caller then runs the
 *   h^eff Trotter step under mask_out, as for TN_MODE_QT).
 * TN_MODE_QSD_SHIFT (MPS): per channel in channel order,
 *   psi <- (1 + dW_k sqrt(gamma_k)(L_k - l_k)) (1 + dt gamma_k (conj(l_k) L_k - |l_k|^2/2)) psi;
 *   same rnd layout as TN_MODE_QSD.
 * TN_EINVAL (before anything runs) when dt is negative or not finite, a uniform of rnd lies
 * outside [0, 1] or a normal is not finite. */
int apply_jumps(void* s, int mode, double dt, const double* rnd, int noise_kind,
                int* jumped_out, unsigned char* mask_out);

/* Correlation matrix C_ij = <c_i^+ c_j> (Sec. 2.1) with the Jordan-Wigner string,
 * by exact contraction of each instance.
 * normalize (MPS): 1 -> <psi|O|psi>/<psi|psi>; 0 -> <psi|O|psi> (the linear QSD estimator of
 * Sec. 4.2, histories not renormalized); 2 -> as 0 per instance (C_each, C_var), but C_mean is
 * the ratio sum_b <psi_b|O|psi_b> / sum_b <psi_b|psi_b>; any other nonzero value acts as 1.
 * MPDO: Tr(rho O)/Tr rho; PURIFIED: Tr(X X^+ O)/Tr(X X^+) (normalize ignored).
 * C_mean: L*L complex, batch mean (row i = c_i^+).  C_var: L*L doubles or NULL, the sample
 * variance of the per-instance values C_b (those C_each holds) with divisor B - 1, around their
 * arithmetic batch mean: sum_b |C_b - mean|^2 / (B - 1), 0 when B = 1; with normalize 2 it is
 * still taken around the arithmetic mean of the linear values, not around the ratio C_mean.
 * sqrt(C_var / B) is the statistical error of eq. ErrorCLT (Sec. 4.1).
 * C_each: B*L*L complex or NULL.  norm_out: B doubles or
 * NULL: <psi|psi> (MPS, PURIFIED) or Tr rho (MPDO), including exp(lognorm). */
int measure_corr(void* s, int normalize, double* C_mean, double* C_var, double* C_each,
                 double* norm_out);

/* ---- asynchronous measurement -------------------------------------------- */

/* The same measurement as measure_corr, overlapped with the steps that follow it.
 * tn_measure_async_bytes: size of a second caller-owned device buffer (256-byte aligned) that
 *   holds a snapshot of the state (tensors, bond weights, dims, log-norms), the measurement's own
 *   workspace and its outputs; 0 for a null handle.
 * tn_measure_async_enable: hand that buffer to the state (the library neither frees nor resizes
 *   it) and create the library's measurement stream (default priority).  TN_ENOMEM if bytes is
 *   below tn_measure_async_bytes, TN_EINVAL on a null or misaligned buffer or while a
 *   measurement is outstanding.
 * measure_corr_start: copy the state, in the order of the work queued on the state's stream,
 *   into the snapshot and launch the measurement of the snapshot on the measurement stream;
 *   returns without waiting.  Later tebd_step / apply_jumps calls evolve the live state
 *   meanwhile.  normalize as for measure_corr.  At most one measurement is outstanding:
 *   TN_EINVAL if one is, or if the buffer was never given.
 * measure_corr_finish: wait for the outstanding measurement and copy its results out, with the
 *   meaning and layout of measure_corr's outputs (C_mean required, the others may be NULL);
 *   TN_EINVAL if none is outstanding.  The results equal those measure_corr would have
 *   returned at the time of measure_corr_start, bit for bit. */
size_t tn_measure_async_bytes(const void* s);
int tn_measure_async_enable(void* s, void* buf, size_t bytes);
int measure_corr_start(void* s, int normalize);
int measure_corr_finish(void* s, double* C_mean, double* C_var, double* C_each, double* norm_out);

/* ---- measurement without device allocation --------------------------------- */

/* For callers that cannot allocate device memory or hand the library a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The same measurement as measure_corr, same arguments, outputs and errors, bit for bit the same
 * results, but the sweep's workspace (right environments, left strings, GEMM temporaries) is a
 * static device array of TN_SCRATCH_BYTES inside the library instead of the arena's workspace
 * region; the instances are measured in groups of as many as that array holds.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and creates nothing.
 * Every state on one GPU shares that GPU's one array, which keeps the last call's contents
 * (the sweep writes every entry it reads, so nothing needs clearing): calls that overlap on one
 * GPU, from two threads or on two streams, race and must not be made.
 * TN_ENOMEM when one instance's workspace exceeds TN_SCRATCH_BYTES (e.g. MPS, FP64, L = 64,
 * chi = 256: 272 MB); TN_EHIP if the array's device address could not be looked up at mps_alloc. */
#define TN_SCRATCH_BYTES ((size_t)128 << 20)
int measure_corr_noalloc(void* s, int normalize, double* C_mean, double* C_var, double* C_each,
                         double* norm_out);

/* Release the handle (not the arena). */
int mps_free(void* s);

/* Thread-local description of the last error ("" if none). */
const char* mps_last_error(void);

/* ---- state I/O: checkpoint / resume and test injection ------------------- */

/* Capacity (in complex numbers) of the tensor buffer of one instance, and in
 * doubles of its bond-weight buffer. */
size_t mps_instance_tensor_capacity(const void* s);
size_t mps_instance_lambda_capacity(const void* s);

/* Read instance `inst`: dims (L+1 ints, dims[0] = dims[L] = 1), tensors packed
 * site after site (chi_l*d_i*chi_r complex each), lambdas packed bond after bond
 * (dims[b+1] doubles each), lognorm and accumulated truncation weight. */
int mps_get_instance(const void* s, int inst, int* dims, double* tensors, double* lambdas,
                     double* lognorm, double* trunc);

/* Overwrite instance `inst` with the same packed layout as mps_get_instance.  Each inner bond
 * dimension dims[b] must lie in 1 .. min(chi_max, d_0 ... d_{b-1}, d_b ... d_{L-1}) (products of
 * the local dimensions left and right of the bond: the largest Schmidt rank the bond can carry,
 * which bounds the per-bond workspace); TN_EINVAL otherwise, and also when a tensor entry or the
 * lognorm is not finite or a bond weight is negative or not finite. */
int mps_set_instance(void* s, int inst, const int* dims, const double* tensors,
                     const double* lambdas, double lognorm);

/* Copy instance src over every other instance (device to device). */
int mps_replicate(void* s, int src);

/* ---- host-side gate builder (no device work) ----------------------------- */

/* Gate of bond b for time tau, as used by tebd_step: 4x4 exp(-i h^eff_b tau) for
 * kind MPS / PURIFIED (before embedding), 16x16 exp(l_b tau) for MPDO in the
 * basis (m_b, m_{b+1}).  out: 16 or 256 complex. */
int tn_gate(int kind, const tn_model* model, int bond, double tau, double* out);

/* ---- autotuner -------------------------------------------------------------- */

/* For n <= 128 the Householder reduction has two variants (0: FP64 MFMA block columns, run as a
 * head launch down to order 64 and a tail launch for the rest; 1: wave tiles, one launch).  The
 * first tebd_step of a state times both, per bucket size class (tn_buckets), on the Gram
 * matrices of the first chunk of that class (median of three) when that chunk holds at least
 * 2048 items, and takes the wave-tile kernel for the class only when it is more than 5 % faster;
 * classes with smaller chunks keep kernel 0 untimed, so the choice does not follow timing noise.
 * tn_tuning reports the choice of the largest class timed (variant_out, may be NULL) and its
 * median times in ms (ms_out[2], may be NULL; zero before tuning or when n > 128); set_variant 0
 * or 1 sets every bucket's choice, -1 only reports.  Returns TN_OK or TN_EINVAL. */
int tn_tuning(void* s, int set_variant, int* variant_out, float* ms_out);

/* ---- bond-size buckets ------------------------------------------------------ */

/* The items of a layer (Sec. 2.3: every bond of one parity of every instance) are formed into
 * chunks bucket by bucket: the bond positions of a parity are grouped by the order their Gram
 * matrix can reach under chi_max (the largest bond dimensions the chain allows): <= 64, <= 128,
 * <= 256, larger; largest first.  A chunk holds the instances of one bucket's bonds (bond-major),
 * its per-item workspace strides and its kernel choices follow that bucket's largest shape, and
 * its Householder kernel is the autotuner's choice for the bucket's size class (timed on the
 * first chunk of that class, see tn_tuning).  Results do not depend on the bucketing beyond the
 * order of roundings.  on = 1 (the default) buckets the layers with at least as many items as the
 * device has compute units and sends a smaller layer out whole (it is latency-bound: one launch
 * sequence instead of several in a row); on = 2 buckets every layer; on = 0 forms chunks from all bonds of the layer
 * in instance order (sized for the state's largest shape); -1 only reports.  Chunks go to the
 * library's two streams by the work already queued on each (items x order^3).  count (may be NULL) receives the
 * number of buckets of the parity (at most 4); nmax, nbonds, hvar (4 ints each, may be NULL)
 * their largest Gram order, their number of bond positions and their Householder variant.
 * Returns TN_OK or TN_EINVAL. */
int tn_buckets(void* s, int on, int parity, int* count, int* nmax, int* nbonds, int* hvar);

/* ---- graph replay --------------------------------------------------------- */

/* tebd_step replays one captured HIP graph per schedule, Trotter order and masking (all layers
 * of one step, kernel launches only; a masked step reads the mask from a fixed arena slot that
 * the call refills first, so one graph serves every mask) while timing is off and the stream
 * given to mps_alloc is a created (non-null) stream; otherwise it launches eagerly.  Both give
 * identical results.
 * on = 0 switches replay off and releases the captured graphs; on = 1 (the default) allows it.
 * Returns TN_OK or TN_EINVAL (null handle). */
int tn_graph_enable(void* s, int on);

/* ---- stream overlap ------------------------------------------------------- */

/* When a layer has more items than one workspace chunk, the arena holds two workspace slots and
 * the library owns a second stream (default priority): chunks alternate between the stream given
 * to mps_alloc and that stream, forked after the work already queued and joined back before the
 * layer's reduction, so kernels of different chunks can share the compute units.  Results do not
 * depend on it (every item is computed the same way).  on = 0 keeps every chunk on the caller's
 * stream; on = 1 (the default) allows the overlap.  Returns TN_OK or TN_EINVAL (null handle). */
int tn_overlap(void* s, int on);

/* ---- precision of the Theta contraction ---------------------------------- */

/* TN_SPLIT forms Theta~ = G (B_b B_{b+1}) (eq. Theta) by default (bits = 32) on the FP32 matrix
 * cores from the complex64 site tensors, with FP32 sums per 8-deep k-chunk added in FP64.  bits =
 * 64 forms it on the FP64 matrix cores instead, where the products of complex64 values are exact
 * and only the FP64 sums round; the split path's error is then that of its complex64 storage.
 * Either way Theta~ is kept in FP64 for the Gram matrix and the split, and the gate is applied in
 * FP64.  The choice matters where the truncation at a binding chi amplifies rounding (saturated
 * states from physical evolution).  TN_FP64 always contracts in FP64 (bits = 32 is refused
 * there).  Results are deterministic for either choice.  Returns TN_OK or TN_EINVAL. */
int tn_theta_precision(void* s, int bits);

/* ---- Trotter schedule ----------------------------------------------------- */

/* Selects how tebd_step applies a Trotter step (both give the same Trotter product, Sec. 2.3):
 * TN_SCHED_LAYER (default): every bond of one parity of every instance is one independent
 *   update (Hastings form, Lambda_{bond-1} as the left environment); exact canonical form is
 *   kept for unitary gates.
 * TN_SCHED_SWEEP: the paper's sequential sweep in the mixed decomposition (eq. MPSMixte):
 *   each two-site SVD is taken on a block holding the orthogonality centre, without Lambda
 *   weights, so the truncation is optimal for any gate; the centre moves by SVD shifts with
 *   the identity gate (eq. ShiftCenter).  Passes alternate direction starting left to right;
 *   before each gate the centre is shifted onto the bond; after the last pass it returns to
 *   site 0, so between steps every tensor but site 0 is right-canonical (eq. GaugeR) and the
 *   state has the same storage form under both schedules.  Parallel over instances only:
 *   about 2(L-1) (order 1) or 4(L-1) (order 2) dependent launch sequences per step.
 * Returns TN_OK or TN_EINVAL (null handle, unknown schedule). */
int tn_schedule(void* s, int schedule);

/* ---- eigensolver path counters ------------------------------------------- */

/* Split precision with n <= 128 and chi <= 64 takes the tridiagonal eigenvectors from bisection
 * and twisted factorization.  An item whose kept eigenvalues are closer than 1e-11 lambda_max (a
 * degenerate multiplet) or whose factorization overflows takes them from inverse iteration
 * instead (a tridiagonal that is not finite or has no positive eigenvalue from implicit QL);
 * an item with two adjacent kept eigenvalues closer than 1.1e-7 sqrt(lambda_p lambda_q) (where
 * the loss of orthogonality weighted by the two singular values reaches 1e-9), and every item of
 * the former kind, has its vectors re-orthogonalized.  tn_stats reports how many two-site updates took each
 * route since mps_alloc or the last reset (either output may be NULL); reset = 1 zeroes both
 * counts after reading them.  Other precisions and shapes count nothing.  Returns TN_OK,
 * TN_EINVAL (null handle) or TN_EHIP. */
int tn_stats(void* s, int reset, long long* cluster_items, long long* reorthogonalized_items);

/* ---- kernel timing (HIP events on the library stream) -------------------- */
#define TN_K_THETA   0  /* Theta formation + gate */
#define TN_K_GRAM    1  /* weighted Gram matrix */
#define TN_K_HETRD   2  /* Householder tridiagonalization */
#define TN_K_STEQR   3  /* tridiagonal eigenvalues (QL, or bisection in split mode) + rank selection */
#define TN_K_VECS    4  /* eigenvectors: rotations + back-transformation */
#define TN_K_SPLIT   5  /* split / store */
#define TN_K_MEASURE 6  /* measurement sweep */
#define TN_K_JUMPS   7  /* dissipative step */
#define TN_K_COUNT   8

/* Enable (1) or disable (0) per-kernel event timing; enabling resets the totals. */
int tn_prof_enable(void* s, int on);
/* Total milliseconds and launch count recorded for a kernel id since enabling (launches on both
 * streams; with two streams, concurrent launches each count their full duration). */
int tn_prof_query(void* s, int kernel_id, double* total_ms, long long* launches);
/* Wall milliseconds since enabling during which at least one launch of the kernel id was running
 * (union of the launch intervals of both streams).  Returns TN_OK or TN_EINVAL. */
int tn_prof_busy(void* s, int kernel_id, double* busy_ms);

#ifdef __cplusplus
}
#endif
#endif /* TEBD_H */
