/*
 * msgfem.h - C ABI of the MI355X (gfx950) local spectral stage of MS-GFEM
 * with A-harmonic local spaces (Benezech, Seelinger, Bastian, Butler,
 * Dodwell, Ma, Scheichl: "Scalable multiscale-spectral GFEM with an
 * application to composite aero-structures").
 *
 * The library computes, for a batch of oversampled subdomains Omega_j^* of a
 * structured hexahedral laminate mesh:
 *   - the Q1 anisotropic-elasticity stiffness a_{Omega*} (Sec. 2, eq. for a_D),
 *     the DoF classes B1/B2/B3 (Sec. 4.3) and the smooth partition of unity
 *     mu_j (Sec. 4.2)                                    -> msgfem_assemble_local
 *   - the n_ev smallest eigenpairs of the A-harmonic GEVP (Sec. 3.3; matrix
 *     form Sec. 4.3), solved through the interior Schur complement
 *                                                        -> msgfem_local_eigs
 *   - building blocks of the same operators (stiffness / PoU products and the
 *     interior solves) for particular functions and checks -> msgfem_local_apply
 *
 * Conventions
 *   - Units mm, N, MPa.  Mesh node id i + (nx+1)*(j + (ny+1)*k); element id
 *     i + nx*(j + ny*k); DoF id 3*node + component.
 *   - Every array marked "device" is a device pointer owned by the caller
 *     (e.g. allocated by PyTorch); the library never allocates device memory
 *     in these calls.  "host" arrays are read during the call only.
 *   - Every compute call is asynchronous on the caller's HIP stream, passed as
 *     `void *stream` (a hipStream_t; NULL = the default stream).  The return
 *     value reports argument and launch errors only; device-side outcomes are
 *     written to the caller's device `status` array (bit flags, below) and are
 *     valid after the stream is synchronised.
 *   - Inputs are never modified.  No exceptions cross the ABI.
 *   - Threads: different plans (and coarse stores) may be used from different
 *     host threads at the same time, each on its own stream; the library's
 *     one-time set-up runs once, whichever thread calls first.  Calls on
 *     one plan must not overlap.
 *
 * Return codes: MSGFEM_OK (0), MSGFEM_EARG (-1) bad argument,
 * MSGFEM_EHIP (-2) HIP error, MSGFEM_ESIZE (-3) unsupported size.
 * The message of the last failure of a plan: msgfem_plan_error().
 *
 * Status bits (device int32 per batch box): 1 = not converged within maxit
 * (best iterate returned), 4 = a pivot of a local factorisation was not
 * positive, 8 = non-finite value met, 16 = every computed eigenpair passed
 * the threshold of msgfem_select_modes.
 */
#ifndef MSGFEM_H
#define MSGFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSGFEM_OK 0
#define MSGFEM_EARG (-1)
#define MSGFEM_EHIP (-2)
#define MSGFEM_ESIZE (-3)

typedef struct msgfem_plan msgfem_plan;

/* Structured laminate mesh (Sec. 2, Sec. 5.1).  All pointers are device. */
typedef struct {
  int32_t nx, ny, nz;        /* elements per axis */
  int32_t n_mat;             /* rows of `materials` */
  const double *node_xyz;    /* [(nx+1)(ny+1)(nz+1)][3] node coordinates */
  const int32_t *elem_mat;   /* [nx*ny*nz] material row of every element */
  const double *materials;   /* [n_mat][10]: E1,E2,E3,G12,G13,G23,nu12,nu13,nu23
                                in the material frame and the ply angle in
                                degrees (rotation about +z, fibre axis
                                (cos t, sin t, 0)) */
  const uint8_t *dirichlet;  /* [3*n_nodes] 1 = DoF clamped to zero (Gamma_D) */
} msgfem_mesh;

/* Overlapping domain decomposition (Sec. 3.1, 3.3).  Host pointers.
 * Omega_j = core grown by `overlap` element layers, Omega_j^* = Omega_j grown
 * by ovs[j] further layers, both clipped to the mesh (the paper's o^* is
 * overlap + ovs[j]).  Every subdomain takes part in the partition of unity;
 * only the batch is solved. */
typedef struct {
  int32_t nsd;
  const int32_t *cores;      /* [nsd][6] element box lo_x,lo_y,lo_z,hi_x,hi_y,hi_z, [lo,hi) */
  int32_t overlap;           /* o >= 1 */
  const int32_t *ovs;        /* [nsd] oversampling layers >= 0 */
} msgfem_decomp;

/* Eigensolver options. */
typedef struct {
  double shift;     /* s > 0 of the shifted pencil M x = nu (S + s M) x (default 1) */
  double tol;       /* residual tolerance on rho (default 1e-6) */
  int32_t maxit;    /* LOBPCG iteration cap (default 200) */
  int32_t block;    /* block width k >= max n_ev (0: max(2 n_ev, n_ev + 8) rounded up to 8); at most 32.
                       With some n_ev > 32 the block is 32 (0 or 32 accepted) and the
                       pairs come in deflated rounds of 24 (see msgfem_local_eigs) */
  int32_t precision;/* 0 = FP64 throughout.
                       1 = mixed: the preconditioner solve (A + s D A D)^{-1}
                       reads an FP32 copy of its factor (FP64 arithmetic); the
                       operator itself (SpMM, the extension and adjoint solves
                       with A11), the Gram matrices, Rayleigh-Ritz, update and
                       residuals stay FP64, so the eigenpairs and residuals are
                       those of the FP64 pencil and only the search directions
                       change (no restart).  ops_bytes grows by the FP32 copy.
                       2 = FP32 operators first (A-harmonic GEVP only): SpMM and
                       all block solves read FP32 copies of the stencil and
                       factors (FP64 arithmetic and dense steps) until every
                       active box has rho <= max(1e-4, 100 tol) (or the largest
                       rho stops halving over two iterations, or after 30
                       iterations), then the block is re-imaged with the FP64
                       operators and the iteration finishes in FP64, so the
                       returned residuals are FP64 residuals */
  int32_t geneo;    /* 0: A-harmonic GEVP on Omega_j^* (Sec. 3.3); 1: classic GenEO GEVP
                       a_{Omega_j}(phi, v) = lambda a_{Omega_j}(Xi phi, Xi v) on Omega_j
                       itself (Sec. 3.2; oversampling ignored), unknowns on every
                       non-Dirichlet DoF, preconditioned by (A + s D A D)^{-1} */
  uint64_t seed;    /* seed of the random start block */
} msgfem_eig_opts;

typedef struct {
  int64_t ops_bytes;    /* device bytes of the assembled-operator buffer */
  int64_t work_bytes;   /* device bytes of the eigensolver workspace */
  int64_t n_eval;       /* sum over the batch of n_ev (length of evals, resid) */
  int64_t n_evec;       /* sum over the batch of n_dof(box)*n_ev(box) */
  int64_t n_dof;        /* sum over the batch of n_dof(box) = 3 * box nodes */
  int32_t block;        /* block width k in use */
  int32_t n_box;        /* batch size */
} msgfem_sizes;

/* Per-box geometry and buffer offsets, for callers that read the assembled
 * operators (layouts documented in msgfem_plan_box). */
typedef struct {
  int32_t sd;                  /* subdomain id */
  int32_t mx, my, mz;          /* box node dims (Omega_j^* node box) */
  int32_t g0[3];               /* global node index of the box's first node */
  int32_t n_nodes, n_dof, n_ev;
  int32_t n1, n2, n3;          /* sizes of B1, B2, B3 (computed on the host from geometry) */
  int64_t stencil_off;         /* byte offset in ops of the stencil:
                                  double [27*9][n_nodes], entry
                                  ((nb*9 + 3*cr + cc)*n_nodes + node), nb = (dx+1)+3(dy+1)+9(dz+1):
                                  a_{Omega*}(phi_{node,cr}, phi_{node+d,cc}) */
  int64_t cls_off;             /* byte offset of uint8 [n_dof] class 1/2/3 */
  int64_t mu_off;              /* byte offset of double [n_dof]: mu_j on B1, 0 elsewhere */
  int64_t vec_off;             /* element offset of this box in block vectors [n_dof][k] */
  int64_t evec_off;            /* element offset in evecs: [n_dof][n_ev] row-major */
  int64_t eval_off;            /* element offset in evals / resid */
} msgfem_box_info;

/* Create a plan for one mesh, one decomposition and a batch of subdomains.
 * batch[nb] are subdomain ids, n_ev[nb] the number of eigenpairs of each
 * (1 <= n_ev <= 48).  `opts` may be NULL (defaults).  Host-side only: reads
 * the host arrays, keeps copies of the mesh descriptor's device pointers
 * (which must stay valid while the plan is used).  Returns MSGFEM_EARG for
 * inconsistent geometry (empty interior block, box thinner than 3 nodes). */
int msgfem_plan_create(msgfem_plan **plan, int device, const msgfem_mesh *mesh,
                       const msgfem_decomp *dec, const int32_t *batch, const int32_t *n_ev,
                       int32_t nb, const msgfem_eig_opts *opts);
void msgfem_plan_destroy(msgfem_plan *plan);
const char *msgfem_plan_error(const msgfem_plan *plan);
int msgfem_plan_sizes(const msgfem_plan *plan, msgfem_sizes *out);
int msgfem_plan_box(const msgfem_plan *plan, int32_t b, msgfem_box_info *out);

/* Plan options, set on the host between calls (they apply from the next call).
 *   MSGFEM_OPT_GRAPH: 0 (default) = every LOBPCG iteration of msgfem_local_eigs
 *     is launched kernel by kernel, with one 4-byte read of the active flags
 *     (a stream synchronisation) per iteration.  1 = the iterations after the
 *     first of each deflated round (FP64 operators, search block [X, W, P]) run
 *     as HIP graphs of 4 (first round) or 6 (later rounds) iterations, captured
 *     on the plan's own non-blocking stream on first use and launched on the
 *     caller's stream, with one read of the active count per launch.  A box
 *     that converges inside a launch is retired there and skipped by every
 *     later kernel, so evals, evecs, resid, iters and status are bitwise those
 *     of mode 0.  Iterations near maxit, the FP32 phase of precision 2 and
 *     profiled calls (msgfem_profile) stay eager.  The plan keeps up to 8
 *     instantiated graphs, keyed by the ops, work and status pointers (a call
 *     with other buffers captures again); setting 0 releases them.
 *   MSGFEM_OPT_SPLIT: 1 (default) = a box matrix (A11 or A + s D A D) whose
 *     slowest node-order axis has at least 8 layers is factored by one level
 *     of nested dissection: the middle layer of nodes is a separator, the
 *     layers on either side are two band chains factored and swept
 *     independently (two work units per box in the block solves), and the
 *     separator's Schur complement is a dense block.  0 = every box matrix
 *     is one band.  Both give the same operators up to rounding.  The layout
 *     of the factors changes, so set it right after msgfem_plan_create,
 *     before msgfem_plan_sizes and msgfem_assemble_local (ops_bytes and
 *     work_bytes change).  A coarse store (msgfem_coarse_create) takes the
 *     plans of the default layout.
 *   MSGFEM_OPT_SOLVE: the block-solve family (for both matrices): 0 (default)
 *     = the widest that fits, 1 = vector FMA (bands up to 65 tiles), 2 =
 *     matrix cores, 8 columns per workgroup (v_mfma_f64_4x4x4f64, bands up to
 *     65 tiles), 3 = matrix cores, 16 columns per workgroup
 *     (v_mfma_f64_16x16x4f64, bands up to 31 tiles); a family the bands do not
 *     fit falls back to the next one down.  It fixes the layout of the factor
 *     copies, so set it before msgfem_assemble_local.  Results agree up to
 *     rounding.
 *   MSGFEM_OPT_SPMM: the kernel of the stencil products A X and D A D X on
 *     blocks of whole 8-column groups: 0 (default) = the LDS-staged plane
 *     sweep (a workgroup per box and 8 columns marches through the box's
 *     node planes with three planes of X in LDS) when the batch has at least
 *     256 such workgroups and every node plane fits one LDS tile of 240
 *     nodes, else one thread per node and 8 columns reading X through the
 *     caches; 1 = always the latter; 2 = the plane sweep wherever it applies,
 *     wider planes split into x-tiles.
 *     Results agree up to rounding; it can change between calls.
 *   MSGFEM_OPT_CHOL: how the tile Cholesky of msgfem_assemble_local is
 *     launched: 0 (default) = one workgroup per matrix for all steps when the
 *     matrices of a factorisation number between 3/4 of the device's compute
 *     units and all of them and their bands are at most 24 tiles wide, else a
 *     launch per step; 1 = always a launch per step; 2 = always one
 *     workgroup per matrix.  The factors are bitwise the same; it can change
 *     between calls.
 * msgfem_plan_set_option returns MSGFEM_EARG for an unknown key or value.
 * msgfem_plan_get_option reads an option or one of the counters of the last
 * msgfem_local_eigs call: MSGFEM_INFO_GRAPH_LAUNCHES (graph launches),
 * MSGFEM_INFO_GRAPH_ITERS (iterations they ran), MSGFEM_INFO_GRAPHS_CACHED;
 * MSGFEM_INFO_SPLIT_BOXES: sum over the batch of 1 (A11 split) + 2 (Ahat split);
 * MSGFEM_INFO_SOLVE_FAMILY: the families in use, A11 + 4 Ahat (1 vector, 2
 * matrix cores 8 columns, 3 matrix cores 16 columns); MSGFEM_INFO_MAX_BT_A11,
 * MSGFEM_INFO_MAX_BT_AHAT: the widest band (tiles) of each matrix in the plan. */
#define MSGFEM_OPT_GRAPH 1
#define MSGFEM_OPT_SPLIT 2
#define MSGFEM_OPT_SOLVE 3
#define MSGFEM_OPT_SPMM 4
#define MSGFEM_OPT_CHOL 5
#define MSGFEM_INFO_GRAPH_LAUNCHES 100
#define MSGFEM_INFO_GRAPH_ITERS 101
#define MSGFEM_INFO_GRAPHS_CACHED 102
#define MSGFEM_INFO_SPLIT_BOXES 103
#define MSGFEM_INFO_SOLVE_FAMILY 104
#define MSGFEM_INFO_MAX_BT_A11 105
#define MSGFEM_INFO_MAX_BT_AHAT 106
int msgfem_plan_set_option(msgfem_plan *plan, int32_t key, int64_t value);
int msgfem_plan_get_option(const msgfem_plan *plan, int32_t key, int64_t *value);

/* Assemble the local operators of every batch box into `ops` (device,
 * ops_bytes): material tensors, partition-of-unity weight sums over all
 * subdomains (Sec. 4.2), block-27 stencils of a_{Omega*} (Sec. 2), DoF
 * classes (Sec. 4.3), mu_j on B1, and the banded Cholesky factors of A11
 * (B1 block) and of A + s D A D on B1 u B2 used by msgfem_local_eigs.
 * status: device int32[nb], overwritten (bit 4 = non-positive pivot). */
int msgfem_assemble_local(msgfem_plan *plan, void *ops, int32_t *status, void *stream);

/* The A-harmonic local GEVP (Sec. 3.3; mixed form and its matrix form Sec.
 * 4.3), reduced exactly to S x = lambda M x on B2 with
 * S = A22 - A21 A11^{-1} A12 and M = E^T (D A D)_{11} E, E = -A11^{-1} A12,
 * and solved as M x = nu (S + s M) x for the n_ev largest nu by LOBPCG
 * preconditioned with the B2 trace of (A + s D A D)^{-1}.
 *   ops   : assembled by msgfem_assemble_local with this plan
 *   work  : device, work_bytes
 *   x0    : NULL (seeded random start) or device block [n_dof][k] per box at
 *           vec_off (values on B2 DoFs are used)
 *   evals : device double[n_eval], lambda ascending per box (eval_off)
 *   evecs : device double[n_evec], per box [n_dof][n_ev] row-major: the
 *           A-harmonic eigenvectors phi = (E x, x, 0) on every DoF of the box,
 *           unit 2-norm, entry of largest magnitude positive
 *   resid : device double[n_eval], rho = |Mx - nu T x| / (|Mx| + nu |T x|)
 *   iters : device int32[nb] LOBPCG iterations (summed over the rounds)
 *   status: device int32[nb], bits ORed in (1 = not converged)
 * With n_ev > 32 on some box (at most 48) the pairs come in deflated rounds:
 * round r finds pairs 24 r .. 24 r + 23 of every box that has them, with a
 * block of 32 kept T-orthogonal (T = S + s M) to the converged pairs of the
 * earlier rounds (classical Gram-Schmidt through the T-Gram cross block,
 * applied to the start block and every preconditioned residual), so the
 * Rayleigh-Ritz step stays 96 x 96.  A round that a later round deflates
 * against converges to rho <= max(1e-4 tol, 1e-10) (the later pairs' residual
 * floor is the earlier pairs' error times the ratio of their nu), or stops
 * six iterations after reaching tol when it stalls short of that.  The work
 * buffer then also holds the four image kinds of every round's converged
 * block. */
int msgfem_local_eigs(msgfem_plan *plan, const void *ops, void *work, const double *x0,
                      double *evals, double *evecs, double *resid, int32_t *iters,
                      int32_t *status, void *stream);

/* msgfem_local_eigs for the boxes a caller selects: mask is a device int32[nb],
 * nonzero = solve that box.  The other boxes are not iterated and their slots
 * of evals, evecs, resid and iters (and their status) are left as they are, so
 * a stored eigen output can be refreshed in place for the boxes whose data
 * changed (offline/online reuse, Sec. 1 and Sec. 6; see msgfem_box_digest).
 * Arguments and errors otherwise as msgfem_local_eigs (MSGFEM_EARG for a null
 * mask). */
int msgfem_local_eigs_subset(msgfem_plan *plan, const void *ops, void *work, const double *x0,
                             const int32_t *mask, double *evals, double *evecs, double *resid,
                             int32_t *iters, int32_t *status, void *stream);

/* Apply one local operator to a block of k columns (box layout [n_dof][k] at
 * vec_off; k must equal the plan's block width, else MSGFEM_EARG):
 *   op 0: y = A x on B1 u B2 (B3 rows/columns removed, 0 on B3)
 *   op 1: y = D A D x (D = diag(mu_j) on B1, 0 elsewhere)
 *   op 2: y = A11^{-1} x on B1, 0 elsewhere (interior solve)
 *   op 3: y = (A + s D A D)^{-1} x on B1 u B2, 0 on B3
 * Entries of x on B3 DoFs are ignored.  Every op uses `work` (device,
 * work_bytes, the same buffer as msgfem_local_eigs; its contents are
 * overwritten).  Reads x, writes y (distinct buffers). */
int msgfem_local_apply(msgfem_plan *plan, const void *ops, void *work, int32_t op, int32_t k,
                       const double *x, double *y, void *stream);

/* msgfem_local_apply without a work buffer, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same operators, kernels, layouts and results as
 * msgfem_local_apply; the scratch it needs (the B3-masked copy of x for ops 0
 * and 1, dofs_total * k doubles; the forward-sweep rows of the block solves for
 * ops 2 and 3, about 2 n_box * ceil(k / 8) * (tile rows + 1) * 256 doubles, and
 * for split boxes 4 n_box * ceil(k / 8) * (separator tile rows + 1) * 256) lives
 * in a static device buffer of msgfem_static_scratch_max() bytes (16 MiB), one
 * per GPU, held until the process ends.  It allocates nothing (no hipMalloc,
 * hipFree or event objects; kernel timing of msgfem_profile is not recorded).
 * Nothing in the buffer needs to start at zero: every call writes the scratch
 * it reads.  All calls on one GPU share that GPU's buffer, so calls that
 * overlap in time on one GPU (two streams, two host threads) race; serialise
 * them.  MSGFEM_ESIZE, before any device work, when a plan needs more scratch
 * than the buffer holds (e.g. the 64-box uniform batch: use msgfem_local_apply
 * with a work buffer there); other errors as msgfem_local_apply. */
int msgfem_local_apply_static(msgfem_plan *plan, const void *ops, int32_t op, int32_t k, const double *x,
                              double *y, void *stream);
int64_t msgfem_static_scratch_max(void);

/* Uniform tractions on the mesh faces (Sec. 2: b(v) = integral of g.v over
 * Gamma_N; the body force is zero).  Host arrays: face[n] with 0..5 =
 * x-, x+, y-, y+, z-, z+ and g[n][3] in MPa. */
typedef struct {
  int32_t n;
  const int32_t *face;
  const double *g;
} msgfem_load;

/* Adaptive local spaces (Sec. 1 and Sec. 5, the threshold t on the reciprocals
 * of the local eigenvalues that selects the eigenvectors of each local space):
 * box j keeps its m_j leading eigenpairs, m_j = the number of its computed
 * eigenvalues with lambda < 1/t (lambda ascending, so 1/lambda_{m_j+1} <= t;
 * the zero eigenvalues of a floating box count while their rounding stays
 * below 1/t).  The comparison is made in double with 1/t rounded once.
 *   evals, evecs: device, as written by msgfem_local_eigs (not modified)
 *   t:            the threshold, > 0 (MSGFEM_EARG otherwise)
 *   evecs_out:    device, msgfem_local_eigs layout: the eigenvectors with the
 *                 columns m_j .. n_ev_j - 1 of every box set to zero, which
 *                 msgfem_coarse_assemble then drops from the coarse basis; it
 *                 may be evecs itself
 *   m:            device int32[nb], m_j per batch box
 *   status:       device int32[nb], bit 16 ORed in where all n_ev_j eigenpairs
 *                 pass (the threshold may need more than were computed). */
int msgfem_select_modes(msgfem_plan *plan, const void *ops, const double *evals, double t,
                        const double *evecs, double *evecs_out, int32_t *m, int32_t *status,
                        void *stream);

/* Error metrics of Sec. 5.3: the relative L2 errors of displacement and
 * strain, e_d = ||u_h - u||_2 / ||u_h||_2 and e_eps = ||eps(u_h) - eps(u)||_2 /
 * ||eps(u_h)||_2, as integrals over the whole mesh (2x2x2 Gauss per element;
 * eps = symmetric gradient, Frobenius norm).
 *   u_ref: device double[n], the reference field u_h (global DoF 3*node+c,
 *          node = i + (nx+1)(j + (ny+1) k), as msgfem_coarse_solve writes u^G)
 *   u:     device double[n], the approximation (e.g. u^G)
 *   n:     3 * the mesh's node count (MSGFEM_EARG otherwise)
 *   out:   device double[6] = [int |u_h-u|^2, int |u_h|^2, int |eps(u_h-u)|^2,
 *          int |eps(u_h)|^2, e_d, e_eps]; a zero reference gives 0 for a zero
 *          difference and +inf otherwise.
 * One workgroup in a fixed order: repeated calls give identical bits. */
int msgfem_error_norms(msgfem_plan *plan, const double *u_ref, const double *u, int64_t n,
                       double *out, void *stream);

/* Offline/online reuse of local spaces (Sec. 1 and Sec. 6: when only some
 * subdomains' data change, their local spaces are recomputed and the others
 * kept).  msgfem_box_digest writes, per batch box, a 64-bit digest of what its
 * local eigenproblem reads once assembled: the stencil of a_{Omega*}, the DoF
 * classes, the partition of unity mu_j, the box geometry and n_ev, salted with
 * the eigensolver options (shift, tol, maxit, block width, geneo, precision,
 * overlap; not the seed).  Equal digests mean the same eigenproblem, bit for
 * bit, so a stored local space can be kept; the digest is the same on every run.
 *   ops:    the plan's assembled operators (after msgfem_assemble_local)
 *   digest: device uint64[nb] */
int msgfem_box_digest(msgfem_plan *plan, const void *ops, uint64_t *digest, void *stream);

/* Copies the eigen output of boxes of plan `src` (e.g. a plan over only the
 * changed subdomains) into the slots of the same subdomains in the eigen output
 * of plan `dst` (e.g. a stored full result), leaving the other boxes as they
 * are.  Both outputs are in the msgfem_local_eigs layout of their plans.
 * boxes: host int32[n_boxes], positions in src's batch of the boxes to copy;
 * NULL copies every box of src (MSGFEM_EARG for a position outside it).
 * MSGFEM_EARG if a source subdomain is not in dst's batch, or its box, n_ev or
 * geneo flag differs, or the plans are on different devices.  All pointers are
 * device; the copies are asynchronous on `stream`. */
int msgfem_merge_eigs(msgfem_plan *dst, msgfem_plan *src, const int32_t *boxes, int32_t n_boxes,
                      const double *src_evals, const double *src_evecs,
                      const double *src_resid, const int32_t *src_iters, double *evals, double *evecs,
                      double *resid, int32_t *iters, void *stream);

/* Size of the caller's coarse buffer and the number N_H of coarse functions
 * (the sum of n_ev over the batch).  The coarse problem needs a batch that
 * lists every subdomain of the decomposition exactly once (MSGFEM_EARG
 * otherwise). */
int msgfem_coarse_sizes(msgfem_plan *plan, int64_t *coarse_bytes, int32_t *n_coarse);

/* MS-GFEM coarse problem (Sec. 3.3; coarse basis of Sec. 4.3).  From the local
 * eigenvectors `evecs` (msgfem_local_eigs) it forms, on every box:
 *   b_{Omega*}: consistent nodal loads of `load` on the box's mesh faces,
 *   psi_j: the particular function, A11 psi = b on B1, 0 on B2 and B3 (zero
 *          Dirichlet data, so the Dirichlet part vanishes),
 *   V_j: mu_j phi_{j,k}, orthonormalised by two Cholesky-QR passes that drop
 *        columns whose orthogonal part is below 1e-12 of the largest norm,
 * and writes the Galerkin system of u^G = u^p + V c (u^p = sum_j mu_j psi_j
 * lifted to the right-hand side):
 *   AH (device, N_H x N_H row-major) = V^T A V over the free DoFs
 *   bH (device, N_H)                 = V^T (b - A u^p)
 * A dropped coarse function gives a unit diagonal entry and a zero right-hand
 * side.  ops/work as for msgfem_local_eigs; coarse: device, coarse_bytes, kept
 * for msgfem_coarse_solve. */
int msgfem_coarse_assemble(msgfem_plan *plan, const void *ops, void *work, const msgfem_load *load,
                           const double *evecs, void *coarse, double *AH, double *bH,
                           int32_t *status, void *stream);

/* Coarse solve: FP64 tile Cholesky of AH, c = AH^{-1} bH (device, N_H), and the
 * MS-GFEM solution on the global mesh uG = u^p + V c (device, 3 * n_nodes,
 * zero on the Dirichlet DoFs); up (nullable, device, 3 * n_nodes) receives
 * u^p.  status[0] gets bit 4 if AH is not numerically positive definite. */
int msgfem_coarse_solve(msgfem_plan *plan, const void *ops, void *work, void *coarse,
                        const double *AH, const double *bH, double *c, double *uG, double *up,
                        int32_t *status, void *stream);

/* Device bytes of the caller's PCG workspace (whole-mesh stencil and vectors). */
int msgfem_pcg_sizes(msgfem_plan *plan, int64_t *bytes);

/* GenEO two-level additive Schwarz preconditioned CG on the whole mesh
 * (Sec. 3.2; the fine reference solve of Sec. 5.3), for comparison with the
 * MS-GFEM coarse approximation.  The plan must be a GenEO plan (opts.geneo =
 * 1) whose batch lists every subdomain, after msgfem_assemble_local,
 * msgfem_local_eigs and msgfem_coarse_assemble (AH is then the coarse matrix
 * A_0 of the GenEO space; its bH is not used).  The preconditioner is
 * M^{-1} = R_0^T A_0^{-1} R_0 + sum_j R_j^T A_j^{-1} R_j with A_j the interior
 * block of Omega_j.  u (device, 3 * n_nodes): initial guess in, solution out
 * (zero on Dirichlet DoFs); iterations stop at |r| <= rtol |b|.  iters, relres:
 * host outputs (the call synchronises the stream).  status[0] = 1 if maxit was
 * reached, bit 4 if A_0 is not numerically positive definite. */
int msgfem_geneo_pcg(msgfem_plan *plan, const void *ops, void *work, void *coarse, const double *AH,
                     const msgfem_load *load, double rtol, int32_t maxit, void *pcg, double *u,
                     int32_t *iters, double *relres, int32_t *status, void *stream);

/* ------------------------------------------------------------------------
 * The coarse problem gathered across plans.  A batch of large oversampled
 * boxes can need more device memory than one plan may take (a 24^3-element
 * box holds about 4 GB of operators and factors), so the local stage streams
 * through plans that each hold part of the subdomains.  A coarse object
 * describes every subdomain of one decomposition (the box of Omega_j^*, or of
 * Omega_j for GenEO) and the layout of a caller-owned device "store"; after
 * each plan's local eigensolve, msgfem_coarse_add puts that plan's share of
 * the coarse problem into the store, and once every subdomain is in, the
 * Galerkin system, the coarse solve and (GenEO) the two-level PCG run from
 * the store alone.  Same mathematics as msgfem_coarse_assemble /
 * msgfem_coarse_solve / msgfem_geneo_pcg (Sec. 3.2, 3.3, 4.3, 4.4).
 * ------------------------------------------------------------------------ */
typedef struct msgfem_coarse msgfem_coarse;

/* Host-side: the boxes of every subdomain (geneo = 1: Omega_j, else
 * Omega_j^*), n_ev[nsd] coarse functions per subdomain (1..32), the overlap
 * pairs and the store layout.  The mesh's device pointers are kept (they must
 * stay valid).  MSGFEM_EARG for inconsistent geometry. */
int msgfem_coarse_create(msgfem_coarse **coarse, int device, const msgfem_mesh *mesh, const msgfem_decomp *dec,
                         const int32_t *n_ev, int32_t geneo);
void msgfem_coarse_destroy(msgfem_coarse *coarse);
const char *msgfem_coarse_error(const msgfem_coarse *coarse);

/* Device bytes of the store, N_H = sum of n_ev, and the number of columns kc
 * the store keeps per subdomain (max n_ev, even). */
int msgfem_coarse_store_sizes(const msgfem_coarse *coarse, int64_t *store_bytes, int32_t *n_coarse, int32_t *n_columns);

/* Where subdomain sd sits: its first DoF in the store's box vectors, its box
 * DoF count and its first row in A^H (any pointer may be NULL). */
int msgfem_coarse_box(const msgfem_coarse *coarse, int32_t sd, int64_t *dof_off, int32_t *n_dof, int32_t *row_off);

/* The coarse data of every box of `plan` (assembled, eigensolved; evecs in
 * its msgfem_local_eigs layout) into the store: the box load b, the
 * particular function psi (A11 psi = b on B1), V_j = mu_j phi orthonormalised
 * by two Cholesky-QR passes with the 1e-12 drop, A V_j, mu_j psi_j and
 * A mu_j psi_j; for a GenEO object also the solve data of the box's interior
 * (Dirichlet) factor, rounded to FP32, for the PCG's local solves.  The plan
 * must describe the same mesh, decomposition and eigenproblem, with the same
 * box and n_ev for each of its subdomains, and (GenEO) the same solve layout
 * as the object, which follows the widest band (MSGFEM_EARG otherwise).
 * Uses the plan's work buffer.  Asynchronous on `stream`; a subdomain added
 * again overwrites its slot. */
int msgfem_coarse_add(msgfem_coarse *coarse, msgfem_plan *plan, const void *ops, void *work, const msgfem_load *load,
                      const double *evecs, void *store, void *stream);

/* AH (device, N_H x N_H row-major) = V^T A V and bH = V^T (b - A u^p) over all
 * subdomains (a dropped coarse function gets a unit diagonal entry and a zero
 * right-hand side).  MSGFEM_EARG until every subdomain has been added. */
int msgfem_coarse_galerkin(msgfem_coarse *coarse, void *store, double *AH, double *bH, void *stream);

/* FP64 tile Cholesky of AH (into the store), c = AH^{-1} bH by a
 * multi-workgroup block solve, and uG = u^p + V c on the global mesh (up, if
 * not NULL, receives u^p); vectors of 3 * mesh nodes.  status[0] gets bit 4
 * if AH is not numerically positive definite. */
int msgfem_coarse_solve_store(msgfem_coarse *coarse, void *store, const double *AH, const double *bH, double *c,
                              double *uG, double *up, int32_t *status, void *stream);

/* Device bytes of the workspace of msgfem_coarse_pcg (whole-mesh stencil,
 * global and box vectors, the local solves' scratch). */
int msgfem_coarse_pcg_sizes(const msgfem_coarse *coarse, int64_t *bytes);

/* GenEO two-level additive Schwarz CG on the whole mesh from a GenEO store
 * (every subdomain added): M^{-1} = R_0^T A_0^{-1} R_0 + sum_j R_j^T A_j^{-1} R_j
 * with A_0 = A0 (msgfem_coarse_galerkin of this object) and the local
 * Dirichlet solves A_j^{-1} from the store's FP32 factor copies (FP64
 * arithmetic; the preconditioner only shapes the iteration).  u: initial
 * guess in, solution out; stops at |r| <= rtol |b|.  iters, relres: host
 * outputs (the call synchronises).  status[0]: bit 1 if maxit was reached,
 * bit 4 if A_0 is not numerically positive definite. */
int msgfem_coarse_pcg(msgfem_coarse *coarse, void *store, const double *A0, const msgfem_load *load, double rtol,
                      int32_t maxit, void *pcg, double *u, int32_t *iters, double *relres, int32_t *status,
                      void *stream);

/* Energy norms with the whole-mesh stencil a completed msgfem_coarse_pcg left
 * in `pcg`: out (device double[2]) = [(u_ref - u)^T A (u_ref - u), u_ref^T A u_ref]
 * over the free DoFs, so e_a = sqrt(out[0] / out[1]). */
int msgfem_coarse_energy(msgfem_coarse *coarse, void *pcg, const double *u_ref, const double *u, double *out,
                         void *stream);

/* Kernel timing.  msgfem_profile(plan, 1) clears the counters and starts
 * recording a pair of HIP events around every launch of the library's hot
 * kernels on the stream the kernel is launched on; msgfem_profile(plan, 0)
 * stops recording.  msgfem_profile_stats synchronises the recorded events and
 * returns, per kernel that ran, the launch count, the summed device time and
 * the summed algorithmic bytes and flops of those launches (the minimal
 * traffic of the algorithm, e.g. the band entries of a factor read once per
 * triangular sweep, not the bytes the hardware moved).  `out` may be NULL to
 * query the count; at most max_out records are written, *n_out is the total. */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double bytes;
  double flops;
} msgfem_kernel_stat;

int msgfem_profile(msgfem_plan *plan, int32_t enable);
int msgfem_profile_stats(msgfem_plan *plan, msgfem_kernel_stat *out, int32_t max_out,
                         int32_t *n_out);

/* ------------------------------------------------------------------------
 * Learned warm start of msgfem_local_eigs (an addition to the method: the
 * paper starts its local eigensolves without prior information).  A small
 * 3D CNN maps the element field of an oversampled box to coefficients C
 * (ng x ne, row-major) of its first ne start vectors in a basis G of ng
 * vectors on B2, the lowest A-harmonic eigenvectors of a homogeneous
 * isotropic reference box of the same node grid (Sec. 4.3 GEVP) made
 * orthonormal on B2.  The start block is X0[:, e] = G C[:, e] on B2 for
 * e < ne and seeded Gaussian columns for e >= ne.  Every call here needs a
 * batch whose boxes share one node grid (MSGFEM_EARG otherwise), ops
 * assembled by msgfem_assemble_local, and is asynchronous on `stream`.
 * ------------------------------------------------------------------------ */

/* Network input of every box: feat (device float[n_box][6][ez][ey][ex],
 * ex = mx - 1 elements along x, ...) with channels, per element, cos 2 theta,
 * sin 2 theta (ply angle), 1 for a ply and 0 for resin (E1 != E2),
 * (ln E1 - ln 1e4) / 2.5 with E1 in MPa, and 2.5 times the mean slopes
 * dz/dx and dz/dy of the element's edges along x and y. */
int msgfem_warm_features(msgfem_plan *plan, const void *ops, float *feat, void *stream);

/* Basis G (device double[n_dof][ng], n_dof of box 0) from the eigenvectors
 * `evecs` that msgfem_local_eigs returned for this plan: the B2 parts of the
 * first ng eigenvectors of box 0 (lambda ascending), orthonormalised over
 * B2 by Gram-Schmidt applied twice; zero rows off B2.  1 <= ng <= n_ev of
 * box 0. */
int msgfem_warm_basis(msgfem_plan *plan, const void *ops, const double *evecs, int32_t ng, double *G,
                      void *stream);

/* Training labels: P (device float[n_box][ng][ng]) = Q Q^T with Q an
 * orthonormal basis (Gram-Schmidt, twice) of G^T X_b, X_b the B2 parts of
 * the first ne eigenvectors of box b in `evecs` (msgfem_local_eigs of this
 * plan); the projector onto the best ne-dimensional approximation of the
 * box's eigenspace in span(G).  G: from msgfem_warm_basis of a box with
 * n_dof_g DoFs, which every box here must have.  Needs ne <= ng,
 * ne <= n_ev and ng * ne <= 8192. */
int msgfem_warm_labels(msgfem_plan *plan, const void *ops, const double *evecs, const double *G,
                       int32_t n_dof_g, int32_t ng, int32_t ne, float *P, void *stream);

/* Start block for msgfem_local_eigs: x0 (device double, box layout
 * [n_dof][k] at vec_off, k the plan's block width) = G coef on B2 for the
 * first ne columns, Gaussian columns from (seed, box, DoF, column)
 * otherwise, 0 off B2.  coef: device float[n_box][ng][ne] (network output).
 * A predicted column that is zero or not finite is replaced by a Gaussian
 * column (the fallback to the random start).  0 <= ne <= k, ng ne <= 12288
 * (the coefficients of a box are staged in LDS); MSGFEM_EARG otherwise. */
int msgfem_warm_start(msgfem_plan *plan, const void *ops, const float *coef, const double *G,
                      int32_t n_dof_g, int32_t ng, int32_t ne, uint64_t seed, double *x0, void *stream);

/* The network: four 3x3x3 convolutions (zero padding 1, strides 1, 1, 2, 2,
 * each followed by ReLU; cin -> width -> width -> width -> width channels)
 * on a d^3 grid, a mean over the last grid, and an affine map to n_out
 * values.  params (device float, n_params): conv weights [width][c_in][27]
 * (tap 9p + 3q + r for the offsets (p-1, q-1, r-1) along z, y, x) and
 * biases of the four layers in order, then the affine weights
 * [n_out][width] and biases [n_out].  Activations and conv weights are held
 * in BF16 (bf16 != 0, rounded to nearest even) or FP32; every sum is FP32.
 * work: device, work_bytes (from msgfem_cnn_sizes for this batch size),
 * holds the activations between msgfem_cnn_forward and msgfem_cnn_backward
 * (same params, batch and bf16). */
int msgfem_cnn_sizes(int32_t cin, int32_t width, int32_t n_out, int32_t d, int32_t batch,
                     int64_t *n_params, int64_t *work_bytes);

/* out (device float[batch][n_out]) for x (device float[batch][cin][d][d][d]). */
int msgfem_cnn_forward(const float *params, int32_t cin, int32_t width, int32_t n_out, int32_t d,
                       int32_t batch, int32_t bf16, const float *x, float *out, void *work,
                       void *stream);

/* grads (device float, n_params, overwritten) of sum(gout * out) with
 * respect to params, from the activations the last msgfem_cnn_forward left
 * in work; the sums over the batch run in a fixed order. */
int msgfem_cnn_backward(const float *params, int32_t cin, int32_t width, int32_t n_out, int32_t d,
                        int32_t batch, int32_t bf16, const float *gout, float *grads, void *work,
                        void *stream);

/* Subspace loss of out viewed as c_b (ng x ne) against the label projectors
 * P_b: loss[b] = |c_b c_b^T - P_b|_F^2 and gout[b] = gscale * 4 (c_b c_b^T -
 * P_b) c_b, its gradient times gscale (1/batch for the mean loss; device
 * float arrays).  It depends on c_b only through c_b c_b^T, so any
 * orthonormal basis of the label subspace has zero loss.  Needs
 * (ng*ne + ng*ng + 256) * 4 <= 65536. */
int msgfem_cnn_loss(const float *out, const float *labels, int32_t ng, int32_t ne, int32_t batch,
                    float gscale, float *loss, float *gout, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on params with gradient grads and moments m, v (device float, n). */
int msgfem_cnn_adam(float *params, const float *grads, float *m, float *v, int64_t n, int32_t step,
                    float lr, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MSGFEM_H */
