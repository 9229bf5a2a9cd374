/*
 * ctm.h -- C interface of the MI355X (gfx950) corner-transfer-matrix library.
 *
 * The library approximates the environment of an infinite PEPS on the square
 * lattice of block sites obtained from the ruby lattice (Sec. II B and the
 * caption of Fig. 2: a 2x2 cell of tensors A, B in a checkerboard, physical
 * dimension d = 2^3 = 8), by the directional corner-transfer-matrix method
 * named in Sec. II C: four chi x chi corners C1..C4 and chi x chi x D^2 edges
 * around the cell (caption of Fig. 3(b)).  From the converged environment it
 * returns the norm per site, nearest-neighbour reduced density matrices and
 * expectation values (Sec. II C, Sec. VI) and the fidelity per lattice site
 * (Sec. III, Eq. "fidelity").
 *
 * Conventions (shared by every entry point):
 *   - PEPS tensors are float64, C order, legs [s, u, l, d, r] (physical index
 *     first; x points right, y points down).  Site (x, y) of an Lx x Ly cell
 *     carries tensor pattern[y * Lx + x].
 *   - One "column step" is the unit of work called a move below: in a move in
 *     direction L/U/R/D the environment absorbs one column (or row) of the cell
 *     and is truncated back to chi.  A sweep is L, R, U, D moves, i.e. 2*Lx +
 *     2*Ly column steps.
 *   - Singular-value decompositions, the truncated pseudo-inverse square roots
 *     of singular values and all normalisations are float64 on the GPU in every
 *     precision mode; `prec` selects only the arithmetic of the bulk tensor
 *     contractions (enlarged corners, half-system products, absorption).
 *
 * Ownership and errors:
 *   - The caller owns the tensor buffers (device memory); they are copied at
 *     ctm_init and never kept.  The caller owns the device workspace, which must
 *     stay alive until ctm_destroy.  Host outputs go to caller buffers.
 *   - All device work is enqueued on the caller's HIP stream.  Calls that
 *     return host data synchronise that stream.
 *   - No call throws.  Each returns a ctm_status; ctm_last_error() gives a
 *     thread-local message for the last non-OK status.  A context is not
 *     thread-safe; distinct contexts are independent.
 */
#ifndef CTM_H
#define CTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_ctx_s* ctm_ctx;

typedef enum {
  CTM_OK = 0,
  CTM_E_INVALID = 1,   /* bad argument, shape or size                      */
  CTM_E_NONFINITE = 2, /* NaN/Inf in an input or in the environment         */
  CTM_E_NOMEM = 3,     /* workspace too small                               */
  CTM_E_NOCONV = 4,    /* not converged within max_sweeps (state is valid)  */
  CTM_E_SOLVER = 5,    /* projector solver failed (e.g. zero half-system)   */
  CTM_E_HIP = 6,       /* a HIP runtime call failed                         */
  CTM_E_STATE = 7      /* call not valid in the context's current state     */
} ctm_status;

typedef enum { CTM_FP64 = 0, CTM_FP32 = 1, CTM_BF16 = 2 } ctm_prec;

/* Direction of a move: the side of the cell whose environment absorbs the
 * next column (row) of sites, as in the directional CTM of Sec. II C. */
typedef enum { CTM_LEFT = 0, CTM_RIGHT = 1, CTM_UP = 2, CTM_DOWN = 3, CTM_SWEEP = 4 } ctm_dir;

typedef enum { CTM_INIT_TRIVIAL = 0, CTM_INIT_DIAG = 1 } ctm_init_kind;

typedef struct {
  int32_t n_inst;          /* independent instances (1 = plain CTM).  Instances
                              with equal (d, D, chi) form a class that is moved
                              in lock-step, every stage one grouped launch over
                              all of its rows (batched form)                      */
  int32_t Lx, Ly;          /* unit cell, 1..4 each                                 */
  int32_t n_tensors;       /* distinct tensors per instance                        */
  const int32_t* pattern;  /* host [Lx*Ly]: tensor id of site (x, y) at y*Lx+x     */
  const int32_t* d;        /* host [n_inst]: physical dimension                    */
  const int32_t* D;        /* host [n_inst]: bond dimension (all legs)             */
  const int32_t* chi;      /* host [n_inst]: environment dimension                 */
  int32_t prec;            /* ctm_prec of the bulk contractions                    */
  int32_t svd_oversample;  /* extra subspace columns p (default 16); with
                              svd_resid_tol = 0 and p >= 8, once chi_eff is known,
                              p - 4 .. p of them, so that the width is a multiple
                              of 16 where that range allows it                   */
  int32_t svd_max_iters;   /* subspace iterations per projector (default 30)       */
  double svd_resid_tol;    /* > 0: Rayleigh-Ritz every iteration, stop when every
                              kept residual < tol*sigma_1 (default 1e-13);
                              0: exactly svd_max_iters iterations, Rayleigh-Ritz
                              only in the last                                    */
  double svd_cutoff;       /* keep sigma_i > cutoff*sigma_1 (default 1e-12)         */
  uint64_t seed;           /* seeds the random start of the subspace iteration     */
  int32_t use_graph;       /* 1: ctm_converge replays one captured HIP graph per
                              sweep (every instance, corner spectra included)
                              after its first sweep; needs svd_resid_tol == 0,
                              timing off and a non-NULL stream (default 0)         */
  int32_t autotune;        /* 1: time the GEMM tile variants on first use of each
                              shape and keep the fastest (default 1)               */
  int32_t concurrent_classes; /* graph mode with several shape classes: 1 makes
                              each class's sweep a concurrent branch of the
                              captured graph (own stream while capturing, own
                              scratch), 0 captures the classes one after the
                              other (default 1)                                   */
  int32_t single_layer;    /* 1: the double-layer contractions of a move (the
                              enlarged corners of Sec. II C, Fig. 3(b), and the
                              edge absorption) take the ket tensor A and the bra
                              tensor one at a time, never forming the D^8 double
                              layer in the contraction: 4 chi^2 d D^6 instead of
                              2 chi^2 D^8 flop per corner, the route to large D
                              (Sec. II D); any precision (default 0)              */
  int32_t complex_tensors; /* 1: the kets are complex (Sec. II A: d D^4 complex
                              coefficients per tensor): A_dev[t] holds float64
                              [d][D][D][D][D][2] (real, imaginary interleaved),
                              B_dev must be NULL (the bra is the conjugate of
                              the ket).  The double layer sum_s A_s (x) conj A_s
                              is stored in a real form: on every doubled leg
                              (x, x') the unitary basis slot (x, x) <- e_(x,x),
                              for x < x' slot (x, x') <- (e_(x,x') + e_(x',x))
                              / sqrt 2 and slot (x', x) <- i (e_(x,x') -
                              e_(x',x)) / sqrt 2 on the down and right legs, the
                              conjugate basis on the up and left legs, which
                              makes every tensor of the network real without
                              changing any contraction.  Spectra, norms and
                              ctm_expect are those of the complex state; the
                              environment (ctm_env_export) is in the real pair
                              basis; density matrices come from
                              ctm_rdm_complex.  Not with single_layer,
                              ctm_fidelity or ctm_boundary_spectrum
                              (CTM_E_INVALID) (default 0)                         */
} ctm_config;

/* Fills *cfg with the defaults above for one instance (caller sets the rest). */
void ctm_config_default(ctm_config* cfg);

/* Bytes of device workspace that ctm_init / ctm_fidelity need for `cfg`. */
ctm_status ctm_workspace_size(const ctm_config* cfg, size_t* bytes);

/*
 * Creates a context: copies the tensors, forms the double-layer tensors
 * a = sum_s A_s (x) conj(B_s) (caption of Fig. 3(a); with B = NULL the bra
 * layer is A itself; with B given it is the mixed network of the fidelity,
 * caption of Fig. 4(a)) and initialises the environment.
 *   A_dev, B_dev: host arrays of n_inst*n_tensors device pointers, instance-
 *                 major, each tensor float64 [d][D][D][D][D].  B_dev may be NULL.
 *   ws_dev, ws_bytes: caller-owned device workspace of at least
 *                 ctm_workspace_size() bytes, 256-byte aligned.
 *   stream:       hipStream_t on which all work is enqueued (NULL = default).
 *   init:         CTM_INIT_TRIVIAL: C = e0 e0^T, T = delta_a0 delta_b0
 *                 delta_uu' (open boundary, boundary ket/bra bonds traced),
 *                 zero-padded to chi.  CTM_INIT_DIAG: C_i = diag(s_i) from
 *                 spectrum_host, T = delta_ab delta_uu', Frobenius-normalised.
 *   spectrum_host: for CTM_INIT_DIAG, float64 [n_inst][Lx*Ly][4][chi_max] with
 *                 chi_max the largest chi; else NULL.
 * Returns CTM_E_NONFINITE if a tensor holds NaN/Inf (nothing is allocated).
 */
ctm_status ctm_init(const ctm_config* cfg, const double* const* A_dev,
                    const double* const* B_dev, void* ws_dev, size_t ws_bytes,
                    void* stream, int32_t init, const double* spectrum_host,
                    ctm_ctx* out);

/*
 * `count` column steps in direction `dir` (Sec. II C; see the conventions
 * above), continuing from where the previous call in that direction stopped;
 * with dir = CTM_SWEEP, `count` full sweeps.  Each column step computes, for
 * every row of the column, the four enlarged corners of the plaquette, the
 * truncating projectors from the float64 truncated SVD of the half-system
 * product, then the renormalised corners and edges, each divided by its
 * Frobenius norm.  Asynchronous.
 */
ctm_status ctm_move(ctm_ctx ctx, int32_t dir, int32_t count);

/*
 * Iterates the directional CTM of Sec. II C to its fixed point: sweeps until
 * the largest l1 change of the normalised corner spectra sigma(C)/sum
 * sigma(C), over all corners and positions of an instance, is below tol, or
 * max_sweeps sweeps were done (the corner spectra as the convergence
 * measure of the environment are this library's reading; the paper gives
 * none).  The change is read back to the host every check_every sweeps; an
 * instance stops sweeping at the first check at which its change is below
 * tol (the instances of a class that are still sweeping move together).
 * At each check the projector subspace width follows the kept count
 * (chi_eff + svd_oversample); a check at which the kept count fills the
 * width does not end the run (the width grows first).  The contractions run
 * at the live extent min(chi, width) rounded up to 8: every index beyond it
 * is an exact zero.  sweeps_out, delta_out: host [n_inst] or NULL.
 * Returns CTM_E_NOCONV (state valid) if some instance did not converge.
 */
ctm_status ctm_converge(ctm_ctx ctx, double tol, int32_t max_sweeps,
                        int32_t check_every, int32_t* sweeps_out, double* delta_out);

/*
 * Per-check metrics of ctm_converge as JSON lines, appended to the file at
 * `path` ("-": standard error; NULL: off).  At every check, one line per
 * instance that swept since the previous check: {"inst", "sweep", "delta"
 * (the convergence measure above), "width" (subspace columns), "live_chi"
 * (the live extent), "ms_per_sweep" (host wall time since the previous
 * check per sweep), "kappa" (norm per site, Sec. III; only with flags & 1,
 * at the cost of one norm evaluation), and per cut "chi_eff" (kept singular
 * values of the half-system product, Sec. II C), "discarded" (sum over the
 * subspace's values beyond the kept ones of s_i^2, divided by the sum over
 * all of them: a lower bound on the truncated weight) and "max_resid"
 * (largest kept residual / s_1; -1 where the residuals were not formed),
 * each an object {"L": [...], "R": [...], "U": [...], "D": [...]} over the
 * move directions, indexed by the site y*Lx+x that owns the cut}.  The file
 * is flushed after every check and closed by ctm_destroy.
 */
ctm_status ctm_set_metrics(ctm_ctx ctx, const char* path, int32_t flags);

/* Singular values of the chi x chi corner matrices C1..C4 of Sec. II C
 * (caption of Fig. 3(b)) of instance `inst`, each divided by their sum,
 * float64 [Lx*Ly][4][chi] (position y*Lx+x, corner C1..C4, descending),
 * zero-padded.  Syncs. */
ctm_status ctm_spectra(ctm_ctx ctx, int32_t inst, double* out_host);

/*
 * Gives every corner of instance `inst` new singular values and keeps its
 * singular vectors: C = U S V^T becomes U diag(s) V^T, then divided by its
 * Frobenius norm; the edges are unchanged (the warm-start reading in which
 * predicted corner spectra are put into an environment mid-run, once the
 * kept count has grown).  spectrum_host: float64 [Lx*Ly][4][chi] (position
 * y*Lx+x, corner C1..C4, descending), >= 0; entries past the corner's rank
 * are ignored.  The convergence measure restarts from the new spectra.  Syncs.
 */
ctm_status ctm_set_corner_spectra(ctm_ctx ctx, int32_t inst, const double* spectrum_host);

/* Norm per site kappa = (Z11 Z00 / (Z10 Z01))^(1/(Lx Ly)) of instance `inst`:
 * the cell in its environment, the corners alone, and the two strip pairs
 * joined directly (Sec. III, Eq. "fidelity" and the paragraph after it).
 * 1x1 and 2x2 cells contract Z11 directly; other cells by row transfer, for
 * which the workspace is planned when chi^2 D^(2 Lx + 2) <= 2^28 (else
 * CTM_E_INVALID).  Syncs. */
ctm_status ctm_norm(ctm_ctx ctx, int32_t inst, double* kappa_out);

/*
 * Two-site reduced density matrix of the bond from site (x, y) to its right
 * (vertical = 0) or lower (vertical = 1) neighbour: the two sites with open
 * physical indices in their environment (Sec. II C: local expectation values
 * and nearest-neighbour correlators from the environment; Sec. VI), divided
 * by its trace, not symmetrised.  rho_host: float64 [(s1,s2)][(s1',s2')] (d^2 x d^2, row =
 * ket indices, column = bra indices, first site = left/upper).  herm_defect
 * (may be NULL): ||rho - rho^T||_F / ||rho||_F.  Syncs.
 */
ctm_status ctm_rdm(ctm_ctx ctx, int32_t inst, int32_t x, int32_t y,
                   int32_t vertical, double* rho_host, double* herm_defect);

/* The same for complex kets (complex_tensors = 1): rho_host float64
 * [(s1,s2)][(s1',s2')][2] (real, imaginary interleaved), divided by its
 * trace; herm_defect (may be NULL): ||rho - rho^H||_F / ||rho||_F.  The
 * physical pairs are contracted in the real pair basis of the legs and
 * transformed back.  CTM_E_INVALID for a context of real tensors (and
 * ctm_rdm for a complex one).  Syncs. */
ctm_status ctm_rdm_complex(ctm_ctx ctx, int32_t inst, int32_t x, int32_t y, int32_t vertical, double* rho_host,
                           double* herm_defect);

/*
 * Expectation value tr(rho h) of a two-site operator on the same bond, with
 * h_host float64 [(s1,s2)][(s1',s2')] (Sec. II B: H is a sum of such
 * nearest-neighbour terms).  Computed on the device.  Syncs.
 */
ctm_status ctm_expect(ctm_ctx ctx, int32_t inst, int32_t x, int32_t y,
                      int32_t vertical, const double* h_host, double* value_out);

/*
 * Fidelity per lattice site between the states of A_dev and B_dev (Sec. III,
 * Eq. "fidelity"): three CTM runs on the networks A(x)A*, B(x)B* and the mixed
 * A(x)B*, each from the trivial start until converged; then
 *   d = |kappa_AB| / sqrt(kappa_AA kappa_BB), all per site.
 * cfg must describe both tensor sets (n_inst must be 1).  d_out, ln_d_out:
 * host scalars.  sweeps_out (may be NULL): host [3] sweeps of the three runs.
 * If a run does not converge within max_sweeps, d_out, ln_d_out and
 * sweeps_out are still filled (from the last state) and CTM_E_NOCONV is
 * returned.
 */
ctm_status ctm_fidelity(const ctm_config* cfg, const double* const* A_dev,
                        const double* const* B_dev, void* ws_dev, size_t ws_bytes,
                        void* stream, double tol, int32_t max_sweeps,
                        double* d_out, double* ln_d_out, int32_t* sweeps_out);

/*
 * ctm_fidelity for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same three CTM runs and the same result, with the workspace taken
 * from a file-scope device array of ctm_fidelity_noalloc_max_bytes() bytes
 * (64 MiB) that each GPU holds from its first use until the process ends.
 * The configuration's use_graph and autotune are ignored (treated as 0).
 * Returns CTM_E_NOMEM when ctm_workspace_size(cfg) exceeds the array.  All
 * calls on one GPU share its array: calls that overlap in time on the same
 * GPU (other threads, other streams) race and must be serialised by the
 * caller.  Every buffer a call reads is written by that call first.
 */
ctm_status ctm_fidelity_noalloc(const ctm_config* cfg, const double* const* A_dev,
                                const double* const* B_dev, void* stream, double tol,
                                int32_t max_sweeps, double* d_out, double* ln_d_out,
                                int32_t* sweeps_out);
size_t ctm_fidelity_noalloc_max_bytes(void);

/*
 * Boundary density operator and entanglement entropy of half an infinite
 * cylinder of circumference nv (Sec. IV, Eq. "Eq:rho" and the paragraph
 * after it): the reduced density matrix of the half cylinder has the
 * spectrum of sigma_L^T sigma_R, where sigma_L (sigma_R) is the dominant left
 * (right) eigenvector of the transfer matrix around the cylinder,
 * approximated by the CTM edges wrapped around a circle of nv sites.
 *   sigma_L: the left edges T4 of column `column`, rows y = 0 .. nv-1 (edge of
 *            row y mod Ly), each edge's up-side chi leg joined to the
 *            down-side leg of the edge above, the last to the first;
 *   sigma_R: the same ring of the right edges T2 of column `column - 1`.
 * Both act on the D^nv virtual indices (v_0 most significant) of the nv bonds
 * that cross the cut between columns column-1 and column; sigma[(ket),(bra)].
 * The eigenvalues are found by block Lanczos (`block` start vectors, at most
 * `krylov` basis vectors, <= D^nv; krylov = D^nv gives the whole spectrum)
 * on sigma_L^T sigma_R in the sigma_R inner product, which treats sigma_L and
 * sigma_R as symmetric (exactly so for the fixed point; a truncated or
 * unconverged environment deviates at the level of its own asymmetry).  All
 * float64 on the device; the ring applications are GEMMs of the ring state
 * (chi^2 D^nv doubles).  Results are divided by the exact trace of
 * sigma_L^T sigma_R (the ring of the double transfer matrices).
 *   nv: a multiple of Ly.  seed: the Lanczos start vectors.
 *   ws_dev, ws_bytes: device workspace of ctm_boundary_workspace_size bytes.
 *   eig_out: host [nev], the largest eigenvalues divided by the trace,
 *            descending (nev <= krylov; entries past the basis are 0).
 *   resid_out (may be NULL): host [nev], residual norm estimates of the Ritz
 *            pairs, divided by the trace (0 when the basis is complete).
 *   entropy_out (may be NULL): -sum p log p over the returned p > 0 (the
 *            entanglement entropy when nev eigenvalues hold all the weight).
 *   weight_out (may be NULL): sum of the returned p.
 * Returns CTM_E_SOLVER if sigma_R is not positive on a start vector or the
 * trace vanishes.  Syncs.
 */
ctm_status ctm_boundary_workspace_size(ctm_ctx ctx, int32_t inst, int32_t nv, int32_t krylov,
                                       size_t* bytes);
ctm_status ctm_boundary_spectrum(ctm_ctx ctx, int32_t inst, int32_t column, int32_t nv,
                                 int32_t krylov, int32_t block, uint64_t seed, void* ws_dev,
                                 size_t ws_bytes, int32_t nev, double* eig_out, double* resid_out,
                                 double* entropy_out, double* weight_out);

/* The environment of Sec. II C (corners C1..C4 chi x chi, edges T1..T4
 * chi x D^2 x chi) of instance `inst` as float64, in the order C1..C4 then
 * T1..T4, each for positions y*Lx+x, legs clockwise around the site,
 * zero-padded to chi; `bytes` must equal ctm_env_bytes().  Import replaces
 * the environment (e.g. with one computed elsewhere); it resets the
 * projector subspaces (cold start of the next solves, full subspace width
 * and extent).  Both sync. */
size_t ctm_env_bytes(ctm_ctx ctx, int32_t inst);
ctm_status ctm_env_export(ctm_ctx ctx, int32_t inst, void* host_buf, size_t bytes);
ctm_status ctm_env_import(ctm_ctx ctx, int32_t inst, const void* host_buf, size_t bytes);

/* Checkpoint of everything a later sweep of instance `inst` depends on: the
 * environment at its live extent, the previous corner spectra, the kept
 * projector subspaces of every cut with their solver statuses (the warm
 * starts of the next solves), the subspace width and the move cursors.
 * Loading it into a context created with the same configuration and tensors
 * makes the following moves and sweeps bitwise equal to those of the saved
 * context.  The layout is private to this library (a versioned header,
 * then device images); `bytes` must equal ctm_checkpoint_bytes().  Both sync.
 * Load returns CTM_E_INVALID for a checkpoint of another configuration. */
size_t ctm_checkpoint_bytes(ctm_ctx ctx, int32_t inst);
ctm_status ctm_checkpoint_save(ctm_ctx ctx, int32_t inst, void* host_buf, size_t bytes);
ctm_status ctm_checkpoint_load(ctm_ctx ctx, int32_t inst, const void* host_buf, size_t bytes);

/*
 * Kernel-time accounting, enabled (and reset) by ctm_set_timing: enable = 1
 * brackets every column step's phases and every launch of the enlarged-corner
 * double-layer contraction with HIP events on the context's stream; enable = 2
 * only the latter (fewer events in the stream); 0 switches it off.  The events
 * are read, and pending ones dropped, by ctm_get_timing / ctm_set_timing, which
 * then wait for them; nothing waits in between.
 * ctm_get_timing fills v[10]:
 *   v[0] seconds in enlarged corners, v[1] in the projector solver,
 *   v[2] in absorption (zero with enable = 2), v[3] seconds inside the
 *   double-layer contraction launches of the enlarged corners, v[4] number of
 *   those launches, v[5] their algorithmic flop at the live extent
 *   (2 chi_live^2 D^8 per corner), v[6] corner-chain launches, v[7] column
 *   steps timed, v[8] the same flop counted at the configured chi (nominal:
 *   the zero-padded work the live extent skips), v[9] the live extent of the
 *   last timed column step.
 */
ctm_status ctm_set_timing(ctm_ctx ctx, int32_t enable);
ctm_status ctm_get_timing(ctm_ctx ctx, double* v);

/*
 * Launch-variant table (process-wide): per kernel family and operand shape,
 * the tile of the generic GEMM, the split counts of the tall-skinny and
 * split-K products ("gemm", "ts", "splitk"), and the rows per work-group of
 * the bf16 products with float32 output, the enlarged corners' and the
 * absorption's ("corner": 256, 192 or 128 for variants 0, 1, 2; ak / bk mark
 * packed operands; bitwise-equal results).  The project's tuner (paper_1711_04798_amd/tune.py) runs
 * the benchmark workloads with tuning on and saves the table; a later
 * process loads it (ctm_init loads the file named by the environment
 * variable CTM_TILE_TABLE once; the Python binding loads the committed
 * table).  Shapes not in the table use defaults (the generic GEMM still
 * times its tiles on first use when a context's autotune is on; its
 * variants give bitwise equal results).
 *   load: entries of the file (written by save: JSON, one entry per line)
 *         replace those of equal key; *entries_out = entries read.
 *   save: writes every entry; *entries_out = entries written.
 *   tune: on = 1 makes the first launch of every new shape of the split
 *         products and the corner product (outside graph capture) time
 *         each variant on its own operands and store the fastest.  The
 *         split products' variants split the
 *         contraction differently, so results change at the rounding level
 *         with the table (a process with one table is deterministic).
 */
ctm_status ctm_tile_table_load(const char* path, int32_t* entries_out);
ctm_status ctm_tile_table_save(const char* path, int32_t* entries_out);
ctm_status ctm_tile_table_tune(int32_t on);
ctm_status ctm_tile_table_clear(void);

/* Releases the context (not the workspace). */
void ctm_destroy(ctm_ctx ctx);

/* Message for the last non-OK status returned on this thread. */
const char* ctm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CTM_H */
