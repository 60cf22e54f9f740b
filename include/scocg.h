/*
 * scocg -- shifted COCG solver for unperturbed Green's-function columns on MI355X.
 *
 * The library computes, for one real-symmetric real-space finite-difference
 * Hamiltonian H of a transition region, the columns
 *
 *     x^{(k)}_j = [Z_k - H]^{-1} e_j ,   Z_k = E_k + i*eta ,
 *
 * of the unperturbed Green's function (Sec. 3B, Eq. 17), restricted to a set S
 * of output rows (only those elements are kept, Appendix after Eq. A12).  One seed
 * Krylov recurrence per right-hand side e_j serves every energy Z_k: the
 * shifted COCG method with collinear residuals (Appendix, Eqs. A7-A12) and
 * seed switching (Eq. A13).
 *
 * Operator (Sec. 2A, Eqs. 2-4, with the nonlocal Kleinman-Bylander extension):
 *     H = H_kin + diag(V) + sum_a P_a diag(D_a) P_a^T
 * Grid nx*ny*nz, index i = ix + nx*(iy + ny*iz) (each x-y plane contiguous).
 * H_kin is a symmetric stencil of half-width nf along each axis: periodic in
 * x and y, truncated in z (the wavefunction vanishes outside planes 0..nz-1,
 * the finite transition block of Eq. 4):
 *     (H_kin v)_i = sum_{axis} sum_{k=-nf..nf} coef[axis][|k|] v_{i + k e_axis}.
 *
 * Conventions for every entry point:
 *   - Return value 0 = success.  Negative = error, no results:
 *       SCOCG_EINVAL (bad shape, index, non-finite input, Im z <= 0),
 *       SCOCG_ENOMEM (device allocation failed), SCOCG_EHIP (HIP runtime
 *       error), SCOCG_ENOSOLVE (green_columns before a successful solve).
 *     Positive = warning with partial results and per-pair status:
 *       SCOCG_NOT_ALL_CONVERGED, SCOCG_BREAKDOWN.
 *     scocg_last_error() returns a thread-local message for the last failure.
 *   - Complex numbers are two doubles (re, im), interleaved.
 *   - Host arrays passed in are copied during the call; the caller keeps them.
 *   - A handle is not thread-safe; concurrent calls on one handle race.
 */
#ifndef SCOCG_H
#define SCOCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCOCG_OK 0
#define SCOCG_EINVAL (-1)
#define SCOCG_ENOMEM (-2)
#define SCOCG_EHIP (-3)
#define SCOCG_ENOSOLVE (-4)
#define SCOCG_NOT_ALL_CONVERGED 1
#define SCOCG_BREAKDOWN 2

/* precision of the Krylov vectors and of the operator arithmetic */
#define SCOCG_FP64 0   /* complex128 vectors, FP64 stencil and projectors */
#define SCOCG_MIXED 1  /* complex64 vectors, FP32 stencil and projectors; every
                          scalar recurrence, x^{(k)} and the dot accumulation in FP64 */

/* per-pair status */
#define SCOCG_PAIR_CONVERGED 0
#define SCOCG_PAIR_MAXITER 1
#define SCOCG_PAIR_BREAKDOWN 2
#define SCOCG_PAIR_STALLED 4   /* SCOCG_MIXED only: the complex64 recurrence stopped
                                  improving above tol (and, with full = 1, the FP64
                                  true residual still misses tol after refinement) */

/* output element type for scocg_green_columns */
#define SCOCG_C128 0
#define SCOCG_C64 1

typedef struct scocg_ctx *scocg_handle;

typedef struct {
    int64_t nx, ny, nz;  /* grid; nx, ny >= nf; nz >= 1 */
    int32_t nf;          /* stencil half-width, 1..4 (4 = the 25-point star) */
    int32_t n_proj;      /* projector channels per atom, 0..4 (0 = no nonlocal part) */
} scocg_grid;

/*
 * Create a handle: uploads H to the device once.
 *   coef      [3][nf+1] host, Ha: H_kin coefficients along x, y, z.
 *   vloc      [N] host, Ha, local potential (diagonal of H).
 *   n_atoms   number of projector blocks (0 allowed).
 *   atom_ptr  [n_atoms+1] host, CSR offsets (atom_ptr[0] = 0, non-decreasing).
 *   atom_idx  [atom_ptr[n_atoms]] host, grid index of each entry, in [0, N);
 *             an index may not repeat within one atom.
 *   atom_P    [entries][n_proj] host, projector values (row per entry).
 *   atom_D    [n_atoms][n_proj] host, Ha, projector energies.
 *   precision SCOCG_FP64 or SCOCG_MIXED.  With SCOCG_MIXED and the environment
 *             variable SCOCG_PROJ=mfma at create time, the projector contraction
 *             C_a = P_a^T X (in solves and scocg_apply_h) and the application
 *             P_a (D_a C_a) (in scocg_apply_h) run on FP32 matrix cores; by default
 *             both run on the vector ALUs, which is faster for 4 channels.
 *   hip_stream hipStream_t to enqueue on (NULL: the handle creates and owns a
 *             non-blocking stream of default priority).
 *   out       receives the handle (freed by scocg_destroy).
 * The current HIP device at create time is the handle's device.
 */
int scocg_create(const scocg_grid *g, const double *coef, const double *vloc,
                 int32_t n_atoms, const int64_t *atom_ptr, const int64_t *atom_idx,
                 const double *atom_P, const double *atom_D, int32_t precision,
                 void *hip_stream, scocg_handle *out);

typedef struct {
    double tol;          /* stop a pair at ||r^{(k)}|| <= tol (||e_j|| = 1); 0 -> 1e-10 */
    int64_t max_iter;    /* seed iterations cap; 0 -> 100000 */
    int32_t init_seed;   /* index of the first seed energy; -1 -> K/2 */
    int32_t seed_switch; /* 1: switch the seed after it converges (Eq. A13); 0: keep it */
    int32_t full;        /* 1: S = all N rows (full x^{(k)} kept; enables the true residual) */
    int32_t refine;      /* SCOCG_MIXED with full = 1: max refinement passes for pairs
                            whose FP64 true residual misses tol (0 = check only, -1 = skip
                            the check); ignored for SCOCG_FP64.  With the check, a
                            SCOCG_MIXED pair is SCOCG_PAIR_CONVERGED iff its FP64 true
                            residual is <= tol */
    int32_t poll_every;  /* seed iterations between host convergence polls, rounded up to a
                            multiple of 6; 0 -> 18 */
    int32_t use_graph;   /* 1: replay the per-poll iterations as one captured hipGraph */
    int32_t timing;      /* 1: bracket every kernel launch with HIP events and report the
                            summed durations per kernel family (scocg_report.kernel_ms);
                            2: only the r_{n+1} pass (SCOCG_K_UPDATE), the lightest probe.
                            Launches are then direct (use_graph is ignored) */
    int32_t tile;        /* stencil workgroup shape, x-y tile TX x TY and threads per group
                            (0 -> 1 for SCOCG_FP64, 3 for SCOCG_MIXED). SCOCG_FP64: 1 = 16x8/1024, 2 = 16x4/512,
                            3 = 8x8/512, 4 = 16x8/512.  SCOCG_MIXED: 1 = 16x8/1024,
                            2 = 16x4/512, 3 = 8x8/1024, 4 = 8x8/512.  nf < 4 always uses 1.
                            SCOCG_AUTO: autotuned (see below) */
    int32_t zchunk;      /* z planes per stencil workgroup (0 -> chosen from the grid size;
                            SCOCG_AUTO: autotuned) */
    int32_t shift_chunk; /* energies per workgroup of the x^(k), p^(k) update: 1, 4 or 16
                            (0 -> 4; SCOCG_AUTO: autotuned) */
    int32_t conventional; /* 1: the conventional COCG sweep the shifted method is compared
                            with (Sec. 3C): every (energy, column) pair runs its own
                            recurrence, nothing is shared between energies; outputs and
                            report as for the shifted solve */
    int32_t aux_seed;    /* 1: start the seed recurrence at the energy seed_z, which need not
                            be one of z (App., after Eq. A13: switching to an arbitrary
                            point).  It is carried as one extra shift -- its pi follows
                            Eq. A8 like every other shift, it is iterated to tol, and the
                            switch of Eq. A13 leaves it once it has converged -- but its
                            solution is neither returned nor reported.  init_seed is
                            ignored.  Not with conventional = 1 or in scocg_batch_solve */
    double seed_z[2];    /* (re, im) of that energy when aux_seed = 1; Im > 0 */
    int32_t symmetric;   /* 1: use G(S_i, e_j) = G(S_j, e_i) (Z - H is complex symmetric):
                            the column block of columns j0.. updates x^{(k)}, p^{(k)} only on
                            rows i >= j0 and the copy-out fills the other rows from the
                            mirror column -- about half the shift-vector work.  Needs
                            S = the RHS set (s_idx NULL), full = 0, conventional = 0.  The
                            mirrored entries carry the mirror column's error (same tol) */
    int32_t cache_mode;  /* cache policy of the r_{n+1} pass: 0 (default) r_{n-1} loads and
                            r_{n+1} stores nontemporal; 1 r_{n+1} stores ordinary (they stay
                            in the last-level cache for the next mu pass); 2 both ordinary;
                            SCOCG_AUTO: autotuned with the launch shape.  Results do not
                            depend on it */
    int32_t zchunk_mu;   /* z planes per workgroup of the mu pass (0 -> the same as zchunk;
                            SCOCG_AUTO: autotuned after the r_{n+1} pass's shape).  The mu
                            pass fits two workgroups per CU and needs only the forward
                            neighbours, so longer chunks can pay there; the partial sums of
                            (r_n, (z_s - H) r_n) are then grouped differently, which changes
                            their rounding (and possibly the iteration count) only */
} scocg_solve_opts;

/* Autotuning: any of tile, zchunk, zchunk_mu, shift_chunk, cache_mode = SCOCG_AUTO makes
   scocg_solve time short trial runs (16 seed iterations from the initial state of this
   very problem) of each candidate launch shape -- the 4 tile shapes x up to 8 z-chunk
   lengths around the default, then up to 6 z-chunk lengths of the mu pass, then 3 shift
   chunks, then 3 cache policies -- before the solve proper,
   keep the fastest, and
   cache it in the handle for this (column blocks, energies, rows) shape; later solves
   of that shape reuse it.  Trials run outside the timed region (scocg_report.tune_ms
   gives their cost, 0 when cached).
   Persistent records: when the environment variable SCOCG_TUNE_CACHE names a file, a
   shape tuned by scocg_solve is also appended to it as one JSON line, e.g.
     {"arch": "gfx950", "precision": "fp64", "grid": [48, 48, 96], "nf": 4, "atoms": 40,
      "block_width": 8, "blocks": 8, "energies": 128, "rows": 64, "tile": 1,
      "zchunk": 18, "shift_chunk": 16, "cache_mode": 0, "zchunk_mu": 32}
   (on one line), and a solve whose handle has no entry for its shape takes the last
   matching record of the file instead of running the trials (scocg_report.tuned = 0).
   Only lines in the exact form written here are read; records with values outside
   the ranges of the options are ignored; a file that cannot be opened is skipped.
   Appends are single writes in append mode, so processes may share one file.
   scocg_batch_solve tunes per batch and does not use the file. */
#define SCOCG_AUTO (-1)

/* kernel families of one seed iteration (index into scocg_report.kernel_ms) */
#define SCOCG_K_PROJ 0     /* (reported as 0: the projector contraction runs inside SCOCG_K_MU) */
#define SCOCG_K_MU 1       /* stencil pass: partials of (r_n, H r_n) + projector contraction;
                              the same launch runs the control step of iteration n - 1 (but
                              at the start of a poll chunk) and the x^(k), p^(k) update of
                              iteration n - 2 */
#define SCOCG_K_ALPHA 2    /* seed alpha_n, c_n */
#define SCOCG_K_UPDATE 3   /* stencil pass: r_{n+1} (three-term recurrence) + dot partials */
#define SCOCG_K_CONTROL 4  /* beta_n, pi recurrences, convergence, compaction, seed switch:
                              timed only where it runs alone, at the end of each poll chunk */
#define SCOCG_K_SHIFT 5    /* (reported as 0: the x^(k), p^(k) update of iteration n runs in the
                              SCOCG_K_MU launch of iteration n + 2) */
#define SCOCG_K_FAMILIES 6

typedef struct {
    int64_t *iters;      /* [K*R] host or NULL: seed iteration at which pair (k,j) froze */
    double *est_resid;   /* [K*R] host or NULL: recursive ||r^{(k)}_j|| at freeze */
    double *true_resid;  /* [K*R] host or NULL: FP64 ||e_j - (Z_k - H) x|| (NaN if not computed) */
    int32_t *status;     /* [K*R] host or NULL: SCOCG_PAIR_* */
    int64_t seed_iters;  /* out: seed iterations run (max over columns) */
    int64_t n_switches;  /* out: seed switches, summed over columns */
    int64_t refined;     /* out: pairs that went through refinement */
    double solve_ms;     /* out: device time of the solve (first kernel to last, HIP events) */
    int64_t block_iters; /* out: column-block iterations run (sum over blocks of B = columns
                            per block: 8 for SCOCG_FP64, 16 for SCOCG_MIXED) */
    int32_t block_width; /* out: B */
    int32_t n_blocks;    /* out: column blocks */
    double kernel_ms[SCOCG_K_FAMILIES];      /* out (timing != 0): summed launch durations */
    int64_t kernel_launches[SCOCG_K_FAMILIES]; /* out (timing != 0): launches timed */
    int32_t tile_used;   /* out: launch shape of the solve (after autotuning) */
    int32_t zchunk_used;
    int32_t shift_chunk_used;
    int32_t tuned;       /* out: 1 if this call ran the autotuning trials */
    double tune_ms;      /* out: device time of the autotuning trials */
    int32_t cache_mode_used; /* out: cache policy of the r_{n+1} pass (scocg_solve_opts) */
    int32_t zchunk_mu_used;  /* out: z planes per workgroup of the mu pass */
} scocg_report;

/*
 * Solve (Z_k - H) x^{(k)}_j = e_{rhs_idx[j]} for all k < K, j < R (Sec. 3B,
 * Eq. 17; Appendix, Eqs. A7-A13).  Index layout of the report arrays: k*R + j.
 *   K, z      K >= 1 energies, host [K][2] (re, im), every Im z > 0.
 *   R, rhs_idx R >= 1 distinct-or-not grid indices in [0, N), host.
 *   nS, s_idx output rows, host; s_idx = NULL and nS = 0 -> S = rhs set.
 *             Ignored when opts->full = 1 (S = 0..N-1).
 *   opts      NULL -> defaults.  rep may be NULL.
 * Blocks the calling thread until the report is filled (one host
 * synchronisation per convergence poll).  Results stay on the device until
 * scocg_green_columns or the next solve.
 */
int scocg_solve(scocg_handle h, int32_t K, const double *z, int32_t R, const int64_t *rhs_idx,
                int32_t nS, const int64_t *s_idx, const scocg_solve_opts *opts,
                scocg_report *rep);

/* One region of a batched solve: the arguments of scocg_solve for that handle. */
typedef struct {
    int32_t K;              /* energies */
    const double *z;        /* [K][2] host */
    int32_t R;              /* right-hand sides */
    const int64_t *rhs_idx; /* [R] host */
    int32_t nS;             /* rows S (see scocg_solve) */
    const int64_t *s_idx;   /* [nS] host or NULL */
} scocg_problem;

/*
 * Batched shifted COCG over n regions (transition regions of any grid size, energy
 * count and column count; the batched form of Sec. 3B and the Appendix): every
 * kernel family of a seed iteration is ONE launch covering all regions (one device
 * table of per-region arguments; regions that have finished idle at no cost), the
 * host polls all regions together, and use_graph replays the polled iterations as
 * one captured hipGraph.
 *   hs        [n] distinct handles on one device and one stream, same precision and nf.
 *   probs     [n] per-region problem (host arrays, copied during the call).
 *   opts      common options; init_seed must be -1.  One tile shape and one shift
 *             chunk serve the whole batch: SCOCG_AUTO for tile or shift_chunk times
 *             16-iteration trials of the whole batch per candidate before the solve
 *             (scocg_report.tune_ms, every call); each region keeps the z-chunk of its
 *             own plan (zchunk = 0 or SCOCG_AUTO) or the explicit one, and its mu pass
 *             that z-chunk unless zchunk_mu is explicit (SCOCG_AUTO counts as 0 here).
 *   reps      [n] or NULL: per-region reports (solve_ms is the whole batch's device
 *             time; kernel_ms/kernel_launches are the shared launches).
 *   region_ms [n] or NULL: device ms from the start of the batch to the host poll at
 *             which the region had finished (after its refinement, if any).
 * Each handle's result is then read with scocg_green_columns.  Return: the worst
 * per-region code (negative codes abort the whole batch).
 */
int scocg_batch_solve(int32_t n, const scocg_handle *hs, const scocg_problem *probs,
                      const scocg_solve_opts *opts, scocg_report *reps, double *region_ms);

/*
 * Copy the last solve's x^{(k)}_j[S] into dst, layout [K][R][nS] (row-major),
 * element SCOCG_C128 (2 doubles) or SCOCG_C64 (2 floats).  dst is a device
 * pointer (dst_is_device = 1, on the handle's device, inside one allocation of
 * at least K R nS elements, else SCOCG_EINVAL) or host memory.
 * Enqueued on the handle's stream; returns after the copy completes.
 */
int scocg_green_columns(scocg_handle h, void *dst, int32_t dtype, int32_t dst_is_device);

/* Apply y = H x for complex128 device vectors x, y of length N (checking aid). */
int scocg_apply_h(scocg_handle h, const void *x_dev, void *y_dev);

/*
 * scocg_apply_h without any device allocation, for callers that cannot allocate
 * (tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same result, bit for bit, with the workspace -- x in a padded column block, the
 * stencil output block, the projector coefficients, the launch's argument table --
 * taken from a static device array of SCOCG_SCRATCH_BYTES per GPU, which the library
 * holds from its first use on that GPU (scocg_create sets it up) until the process
 * ends.  x_dev, y_dev: complex128 device vectors of length N on the handle's device.
 * The workspace needs about 2 (nz + 2 nf) nx ny 128 bytes plus n_atoms 512 bytes (and,
 * for SCOCG_MIXED, 128 bytes per projector entry for the per-entry products);
 * a larger grid is rejected with SCOCG_EINVAL before any launch.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (two threads, or two
 * streams) race and must be serialised by the caller.  Enqueued on the handle's
 * stream; returns after y is written.
 */
#define SCOCG_SCRATCH_BYTES (64u << 20)
int scocg_apply_h_noalloc(scocg_handle h, const void *x_dev, void *y_dev);

/*
 * Open-boundary matching (Sec. 3B, Eqs. 18-24) and transmission (Sec. 2B, Eq. 14).
 *
 * From the unperturbed Green's function of the isolated transition region on an
 * index list idx = (left block, right block, extra rows) -- the left block being
 * the M rows nearest the left lead (the first principal layer z_0: for half-width
 * nf the first nf x-y planes), the right block the M rows nearest the right lead
 * (z_{m+1}), then L rows anywhere (e.g. a plane whose local density of states is
 * wanted, Sec. 3B after Eq. 24) -- and the two lead self-energies, compute for
 * every energy Z_k:
 *   - the perturbed Green's function G_T(Z_k) on idx x idx: the inverse of Eq. 13
 *     restricted to idx, obtained from Eq. 18 on the boundary rows,
 *         (I - G_bb Sigma_b) G_T(b, :) = G(b, :),  Sigma_b = diag(Sigma_L, Sigma_R),
 *     solved as one 2M x 2M system (the block elimination of Eqs. 19-24 done by
 *     Gauss-Jordan elimination with partial pivoting), and on the extra rows
 *         G_T(l, :) = G(l, :) + G(l, b) Sigma_b G_T(b, :);
 *   - the Fisher-Lee transmission T = Tr[Gamma_L G^a(z_0, z_{m+1}) Gamma_R
 *     G^r(z_{m+1}, z_0)] with Gamma = i (Sigma - Sigma^dagger) (Eqs. 14-16), taking
 *     G^r = G_T(Z_k) and G^a its conjugate transpose;
 *   - the density of states of the extra rows, -Im tr G_T(l, l) / pi.
 *
 * Arguments (all matrices complex128, column-major per energy: element (r, c) at
 * r + ld * c; device pointers are on the handle's device and must lie inside one
 * allocation, else SCOCG_EINVAL):
 *   K          energies, 1..16383.
 *   M          rows per boundary block (>= 1); L extra rows (>= 0); D = 2M + L.
 *   g_dev      [K][D][D] device: G(Z_k)[idx_r, idx_c] at r + D c -- the layout that
 *              scocg_green_columns writes after scocg_solve with rhs_idx = idx and
 *              S = the RHS set (G is complex symmetric, so rows and columns agree).
 *   sig_l_dev  [K][M][M] device: Sigma_L(z_0; Z_k) on the left block's rows.
 *   sig_r_dev  [K][M][M] device: Sigma_R(z_{m+1}; Z_k) on the right block's rows.
 *   gt_dev     [K][D][D] device output, G_T on idx x idx (same layout), or NULL; it
 *              may not overlap an input.
 *   trans      [K][2] host output (re, im of T; im vanishes up to rounding) or NULL.
 *   dos        [K] host output or NULL (0 when L = 0).
 *   phase_ms   [4] host output or NULL: device time of the phases, from HIP events
 *              around each launch -- 0 forming I - G_bb Sigma_b, 1 elimination panels,
 *              2 panel updates of the other columns, 3 output rows, T and DOS.
 * Work runs on the handle's stream; the call returns after it completes.  The
 * handle's operator and last solve are not used or changed.  Device workspace of
 * about 16 K ((2M + 32) (2M + D) + 64 M + 3 M^2 + 2 L M) bytes (plus K D^2 16 bytes
 * when gt_dev is NULL) is allocated for the call.
 * Returns SCOCG_BREAKDOWN (outputs of the affected energies NaN) if the 2M x 2M
 * system of an energy meets a zero pivot.
 */
int scocg_obm(scocg_handle h, int32_t K, int32_t M, int32_t L, const void *g_dev,
              const void *sig_l_dev, const void *sig_r_dev, void *gt_dev, double *trans,
              double *dos, double *phase_ms);

/*
 * Streaming bandwidth probe (a measuring aid: the ceiling the memory-bound passes are
 * compared with).  Runs the access mix of one pass without its arithmetic over three
 * equal arrays carved from buf: mode 0 copies (one read, one write, like a plain copy),
 * mode 1 adds two arrays into the third (two reads, one write: the r_{n+1} pass), mode
 * 2 only reads (the mu pass).  16-byte vectors, nontemporal = 1 with nontemporal loads
 * and stores (as the passes stream r_{n-1} and r_{n+1}).  buf: device memory of the
 * handle's device, `bytes` long (>= 12 KiB; use well beyond the 256 MB last-level
 * cache); its contents are overwritten.  After one warm launch, reps launches are
 * timed with HIP events on the handle's stream; *gbs receives bytes read + written per
 * second / 1e9.
 */
int scocg_stream_probe(scocg_handle h, int32_t mode, int32_t nontemporal, void *buf,
                       int64_t bytes, int32_t reps, double *gbs);

/* Release every device buffer of the handle.  NULL is ignored. */
void scocg_destroy(scocg_handle h);

/* Thread-local description of the last error ("" if none). */
const char *scocg_last_error(void);

/* Size in bytes of the ABI structs, for bindings to check their mirrors:
   which = 0 scocg_grid, 1 scocg_solve_opts, 2 scocg_report, 3 scocg_problem; 0 for
   any other value.  Needs no GPU. */
int64_t scocg_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* SCOCG_H */
