/*
 * nlfem.h - C ABI of the MI355X (gfx950) nonlocal P1 finite-element
 * assembler.
 *
 * The library assembles the stiffness matrix of the approximate bilinear
 * form (Klar, Vollmann, Schulz, "nlfem", arXiv 2207.03921, Sec. 2.2,
 * eq. biFormApprox)
 *
 *   A_h(phi_j, phi_i) = sum_k sum_l int_{T_k} int_{T_l}
 *                       1_{B(x)}(y) Phi_ij(x, y) dy dx,
 *   Phi_ij(x, y) = (phi_i(x) - phi_i(y))^T (Psi(x,y) phi_j(x) - Psi(y,x) phi_j(y))
 *
 * for continuous P1 ansatz functions on a triangulation labelled into the
 * domain Omega (label 1) and the interaction domain Omega_D (label 2)
 * (Sec. 2.2, Assumption 2), together with the load vector (f, phi_i).
 *
 * Conventions shared by all entry points
 *  - All mesh, matrix and vector arrays are DEVICE pointers owned by the
 *    caller; they must stay valid until the work enqueued on `stream`
 *    has completed.  Quadrature tables and polygon directions are HOST
 *    pointers, read during the call.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Every call enqueues its work on that stream and returns without
 *    waiting, except where a call is documented as synchronising.
 *  - Return value: NLFEM_OK (0) or a negative NLFEM_E_* code; the message of
 *    the last failure on the calling thread is returned by
 *    nlfem_last_error().  No call aborts or throws.
 *  - Element vertex order may be clockwise or counter-clockwise.
 *  - A node is a degree of freedom iff it is a vertex of some Omega element
 *    and of no Omega_D element (Sec. 2.2, Fig. 2.1).  Elements with other
 *    labels are ignored (Sec. 2.5 allows marking elements that are not part
 *    of the discretisation).
 *  - The matrix is returned in CSR form (Sec. 1: the Python front end returns
 *    CSR) over n*M rows and n*M columns, n = 1 (scalar) or 2
 *    (peridynamics); row/column n*node + component.  With the
 *    discontinuous ansatz (cfg.ansatz = NLFEM_ANSATZ_DG) over n*3K rows and
 *    columns, row/column n*(3k + a) + component; rows of elements outside
 *    Omega are empty.  Rows of nodes that are
 *    not degrees of freedom are empty.  Column indices ascend within a row;
 *    the pattern holds every entry touched by some interacting element pair,
 *    including numerically zero ones.  Splitting the columns into degrees of
 *    freedom and Omega_D nodes yields the Dirichlet splitting of Sec. 3
 *    (eq. inhomogeneousDirichletData).
 */
#ifndef NLFEM_H
#define NLFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLFEM_ABI_VERSION 5

/* return codes */
enum {
    NLFEM_OK = 0,
    NLFEM_E_INVALID = -1,   /* bad argument: NULL pointer, size <= 0, delta <= 0,
                               weights not summing to 1/2, unsupported option */
    NLFEM_E_MESH = -2,      /* vertex index out of range, zero-area element,
                               an edge shared by more than two elements (the
                               mesh is not conforming, Sec. 2.2 Assumption 2),
                               or a material id outside the material table */
    NLFEM_E_NOMEM = -3,     /* device allocation failed */
    NLFEM_E_HIP = -4,       /* HIP runtime error (message has the HIP text) */
    NLFEM_E_OVERFLOW = -5,  /* a count exceeds 32-bit column indices, an
                               internal capacity or the limit set by
                               nlfem_set_capacity */
    NLFEM_E_MISMATCH = -6,  /* handle built for another mesh or configuration */
    NLFEM_E_NODEVICE = -7   /* no HIP device available */
};

/* kernel functions Psi (Sec. 3.1 and 3.2) */
enum {
    NLFEM_K_CONSTANT = 0,    /* Psi = c                       (s = -1)    */
    NLFEM_K_INV_DIST = 1,    /* Psi = c / |x - y|             (s = -1/2)  */
    NLFEM_K_PERIDYNAMIC = 2, /* Psi = c (x-y)(x-y)^T / |x-y|^3, 2 components */
    NLFEM_K_FRAC_HALF = 3    /* Psi = c / |x - y|^3           (s = 1/2: the
                                fractional-type kernel of Sec. 3.1, constant
                                c_{1/2,delta} = 1 / (pi delta)); needs
                                singular_n > 0 */
};

/* ball approximations 1_{B(x)}(y) for the Euclidean ball of radius delta */
enum {
    NLFEM_A_NOCAPS_BARY = 0,     /* T_l counts for x iff |x - bary(T_l)| <= delta */
    NLFEM_A_APPROXCAPS_POLY = 1, /* regular polygon inscribed in the circle,
                                    T_l n polygon retriangulated (Sec. 2.4.1) */
    NLFEM_A_INF_BALL = 2,        /* the infinity-norm ball {y : |x - y|_inf <= delta}
                                    (Def. 2.5): the square with corners
                                    x + delta (+-1, +-1), T_l n square clipped and
                                    retriangulated like the polygon, which is exact
                                    here; polygon_n and polygon_dirs are unused */
    NLFEM_A_NOCAPS = 3,          /* Def. 2.3: the convex hull of the crossings of
                                    the circle |y - x| = delta with the element
                                    edges; on T_l the hull of its vertices in the
                                    disc and its edge crossings, retriangulated
                                    (Sec. 2.4.1) */
    NLFEM_A_APPROXCAPS = 4       /* Def. 2.4: as NOCAPS plus the centre of every
                                    circular cap (midpoint of each arc inside an
                                    element) */
};

/* arithmetic of the quadrature of non-touching pairs */
enum {
    NLFEM_P_FP64 = 0,   /* everything in FP64 */
    NLFEM_P_MIXED = 1   /* non-touching pairs in FP32 with FP32 accumulation per
                           pair; inclusion tests, polygon clipping, touching pairs
                           and the global sums stay FP64.  The constant kernel
                           under NLFEM_A_NOCAPS_BARY (outer rules of up to 8
                           points, continuous ansatz) has no quadrature loop:
                           its non-touching blocks factor into one-element rule
                           sums over the points' status bits (Sec. 2.3, 2.4.1)
                           and are formed in FP64 in either precision */
};

/* ansatz spaces (Sec. 1, 2.3) */
enum {
    NLFEM_ANSATZ_CG = 0,   /* continuous P1: unknown n*node + component */
    NLFEM_ANSATZ_DG = 1    /* discontinuous P1: three basis functions per
                              element, unknown n*(3k + a) + component for
                              vertex a (stored order) of element k; rows for
                              the elements of Omega.  Every kernel (s <= 1/2,
                              Sec. 2.4.2); with NLFEM_K_FRAC_HALF the
                              edge-touching integrals of functions that jump
                              across the shared edge diverge logarithmically
                              and the value is that of the Gauss rule of
                              order singular_n, as in the paper's DG study */
};

/* pair classes (Sec. 2.3: intersecting pairs are vertex touching, edge
   touching or identical) */
enum { NLFEM_C_FAR = 0, NLFEM_C_VERTEX = 1, NLFEM_C_EDGE = 2, NLFEM_C_IDENT = 3 };

typedef struct {
    int64_t n_vertices;        /* M >= 1 */
    int64_t n_elements;        /* K >= 1 */
    const double *vertices;    /* device, [M][2] */
    const int32_t *elements;   /* device, [K][3] vertex indices in [0, M) */
    const int32_t *labels;     /* device, [K]: 1 Omega, 2 Omega_D, other = ignored */
    const int32_t *materials;  /* device, [K] material ids in [0, n_materials)
                                  of the configuration's material table, or
                                  NULL (all 0); read only when the table is
                                  given (Sec. 1: kernels that depend on
                                  element labels, for interface problems) */
} nlfem_mesh;

/* quadrature rule on the reference triangle {xi >= 0, xi_1 + xi_2 <= 1}
   (Sec. 2.4.1); weights sum to 1/2.  1 <= n <= 16. */
typedef struct {
    int32_t n;
    const double *xi;          /* host, [n][2] */
    const double *w;           /* host, [n] */
} nlfem_rule;

typedef struct {
    int32_t kernel;            /* NLFEM_K_* */
    double c;                  /* kernel constant */
    double delta;              /* horizon > 0 */
    int32_t approach;          /* NLFEM_A_* */
    int32_t polygon_n;         /* polygon vertices (approach POLY), 3..64 */
    const double *polygon_dirs;/* host, [polygon_n][2] unit directions, CCW;
                                  vertex j = x + delta * dir_j */
    nlfem_rule outer;          /* rule for the outer element T_k */
    nlfem_rule inner;          /* rule for the inner element T_l */
    int32_t singular_n;        /* Gauss-Legendre points per direction of the
                                  regularising transforms on touching pairs
                                  (Sec. 2.4.2); 0 = touching pairs use the
                                  product rule with the ball like all others
                                  (Table 1); for INV_DIST and PERIDYNAMIC
                                  (s <= 0) that rule avoids zero division:
                                  point pairs with |x - y|^2 <=
                                  1e-12 min(|det J_k|, |det J_l|), the same
                                  point of both elements, are skipped.
                                  Required > 0 for FRAC_HALF; 0 with a
                                  singular kernel runs in the single-problem
                                  path only (not in batches).  0..32. */
    int32_t precision;         /* NLFEM_P_* */
    int32_t ansatz;            /* NLFEM_ANSATZ_* */
    int32_t n_materials;       /* 0 (no table) or 1..4 */
    const double *material_c;  /* host, [n_materials][n_materials]: the
                                  kernel becomes
                                    Psi(x, y) = material_c[m(x)][m(y)] Psi0(x, y)
                                  with Psi0 the kernel above and m(x) the
                                  material of the element holding x (Sec. 1
                                  and 2.1: label-dependent and non-symmetric
                                  kernels).  A non-symmetric table gives a
                                  non-symmetric matrix; it needs a kernel with
                                  s <= 0 (not FRAC_HALF: the difference of the
                                  two directions is not integrable on touching
                                  pairs) and runs in the single-problem path
                                  (not in batches).  Row i, column j of the
                                  matrix is a(phi_j, phi_i): test function in
                                  the row, trial function in the column. */
} nlfem_config;

typedef struct nlfem_pairs nlfem_pairs;   /* opaque, library-owned */

typedef struct {
    int64_t n_pairs;      /* interacting ordered pairs (k, l), labels in {1,2},
                             at least one of them 1 */
    int64_t n_far;        /* ... of class NLFEM_C_FAR */
    int64_t n_vertex, n_edge, n_ident;   /* ... touching classes */
    int64_t n_dof;        /* degree-of-freedom nodes (DG: 3 x Omega elements) */
    int64_t n_rows;       /* n * n_dof matrix rows that may hold entries */
    int64_t nnz;          /* stored entries of the CSR matrix */
    int64_t n_upper_far;  /* unordered non-touching pairs processed by assemble */
    int64_t n_upper_touch;/* unordered touching pairs processed by assemble */
    int64_t n_nbr;        /* entries of the symmetric neighbour lists
                             S(k) = {l : (k,l) or (l,k) interacts}, summed over k */
    int64_t rebuild;      /* how the last nlfem_build_pairs ran: 0 plain build,
                             1 rebuild with the sizes of the build before it
                             (launched without waiting), 2 such a rebuild found
                             other sizes and was run again as a plain build by
                             the call that checked it */
    int64_t skipped;      /* nlfem_assemble calls on this handle, since it was
                             created, whose work was skipped because they were
                             queued after a rebuild that found other sizes
                             (their val was left unchanged; see nlfem_assemble) */
} nlfem_pairs_info_t;

/* Device memory of handles and batches.  alloc(bytes, stream, ctx) returns
   device memory of the current device, aligned to at least 256 bytes, that
   work enqueued on `stream` may use from then on, or NULL (the calling entry
   point then returns E_NOMEM).  free_(ptr, stream, ctx) gives back a block
   of an earlier alloc with the stream it was allocated on; work the library
   enqueued on that stream before the call may still be using it, so the
   free must be stream-ordered (as torch's caching allocator and
   hipFreeAsync are) or wait for the stream.  Both NULL: hipMalloc/hipFree
   (the default).  A block is always released by the pair it came from,
   even after the hooks were replaced.  Set it before the calls that
   allocate; not thread-safe.  Errors: E_INVALID (exactly one of the two
   functions NULL). */
typedef void *(*nlfem_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*nlfem_free_fn)(void *ptr, void *stream, void *ctx);
int nlfem_set_allocator(nlfem_alloc_fn alloc, nlfem_free_fn free_, void *ctx);

/* Largest number of neighbour-list entries (nlfem_pairs_info_t.n_nbr, the
   size that all other buffers of a handle follow) a plain build may hold;
   past it nlfem_build_pairs returns E_OVERFLOW before allocating them.
   0 = no limit (2^31 - 1 entries, the bound of 32-bit list indices).
   For callers that bound device memory per problem, and to test the
   overflow path.  Not thread-safe.  Errors: E_INVALID (negative). */
int nlfem_set_capacity(int64_t max_entries);

/* ABI version (NLFEM_ABI_VERSION of the built library). */
int32_t nlfem_version(void);

/* Message of the last failing call on this thread; valid until the next
   call on this thread.  Never NULL. */
const char *nlfem_last_error(void);

/* Interaction traversal (Sec. 2.5): finds all interacting element pairs of
   the mesh for `cfg` and the CSR pattern of the matrix.
   Pair (k, l) interacts iff both labels are in {1, 2}, at least one is 1, and
   either (singular_n > 0 and T_k, T_l share a vertex) - class = number of
   shared vertices - or some outer quadrature point x_p of T_k sees T_l
   through the ball approximation (class FAR).  All inclusion decisions are
   taken in FP64 with the same operation order as the plain definition
   (no fused multiply-add), so the pattern does not depend on `precision`.
   *pairs: if NULL a new handle is created; otherwise the given handle is
   rebuilt in place, reusing its device memory when large enough.
   A plain build synchronises with `stream` four times (sizes are needed to
   allocate) and allocates through the hooks of nlfem_set_allocator.  A rebuild of a handle whose last plain build had the same
   numbers of vertices and elements and the same kernel, delta, ball, rules
   and singular flag is launched with that build's sizes and returns without
   waiting; its kernels compare the device-side counts with the expected ones
   and skip their work on a difference.  The next call that uses the handle
   (nlfem_pairs_info, _export, _csr_pattern, nlfem_assemble - after queueing
   its own launches, which skip their work likewise -, nlfem_batch_*) waits
   for the rebuild's counts and, when they differ, runs the plain build (and,
   in nlfem_assemble, the assembly again); nlfem_pairs_info_t.rebuild tells
   which happened.  Until that call the mesh arrays must stay valid, and an
   error of the rebuild (E_MESH, ...) is returned by that call.  A batch
   holding the handle stays valid across rebuilds that keep the sizes; after
   a plain rebuild its runs return E_MISMATCH.
   E_MESH is returned for a vertex index outside [0, M), an element of zero
   area, or an edge shared by more than two elements of labels 1 and 2.
   Errors: E_INVALID, E_MESH, E_NOMEM, E_HIP, E_OVERFLOW, E_NODEVICE. */
int nlfem_build_pairs(const nlfem_mesh *mesh, const nlfem_config *cfg,
                      nlfem_pairs **pairs, void *stream);

/* Counts of a built handle.  Synchronous.  Errors: E_INVALID. */
int nlfem_pairs_info(const nlfem_pairs *pairs, nlfem_pairs_info_t *info);

/* Ordered pair list sorted by (k, l): k[n_pairs], l[n_pairs] (int32) and
   cls[n_pairs] (NLFEM_C_*) device arrays owned by the caller.
   Errors: E_INVALID, E_HIP. */
int nlfem_pairs_export(const nlfem_pairs *pairs, int32_t *k, int32_t *l,
                       int8_t *cls, void *stream);

/* CSR pattern: row_ptr[n*M + 1] (DG: [n*3K + 1]) (int64) and col[nnz]
   (int32), device arrays owned by the caller.  Errors: E_INVALID, E_HIP. */
int nlfem_csr_pattern(const nlfem_pairs *pairs, int64_t *row_ptr, int32_t *col,
                      void *stream);

/* Stiffness matrix values val[nnz] (device, FP64) in the pattern of `pairs`
   (eq. biFormApprox with the local contributions of eq. def:localStiffness):
   non-touching pairs by the product rule with the ball approximation
   (Sec. 2.4.1, eq. discrete-inner), touching pairs of a singular
   configuration by the regularising transforms (Sec. 2.4.2, Alg. 1).
   `mesh` must be the mesh the handle was built from; `cfg` may differ from
   the build configuration only in `c`, `precision` and `singular_n` when
   the latter keeps its zero/non-zero status (E_MISMATCH otherwise).
   Allocates nothing and never synchronises: every call only enqueues
   kernels on `stream`.  Uses workspace held by the handle, so two
   assemblies with the same handle must not overlap in time.
   After a rebuild that returned without waiting (see nlfem_build_pairs),
   the kernels compare the rebuild's device-side counts with the sizes the
   handle had before it; if they differ, the kernels skip their work and
   val is left unchanged.  The next nlfem_pairs_info reports that case
   (rebuild = 2, `skipped` counts such calls); query the sizes there and
   assemble again.  When the rebuild kept its sizes (rebuild = 1), val holds
   the result as always.
   Errors: E_INVALID, E_MISMATCH, E_HIP. */
int nlfem_assemble(const nlfem_mesh *mesh, const nlfem_config *cfg,
                   const nlfem_pairs *pairs, double *val, void *stream);

/* Load vector b[n*M] (DG: b[n*3K]) (device, FP64):
     b_(n i + c) = sum over Omega elements T containing node i of
                   |J_T| sum_p d_p f_c(x_p) phi^_(i)(xi_p)
   (DG: b_(n(3k + a) + c) = |J_k| sum_p d_p f_c(x_p) phi^_a(xi_p) for the
   elements of Omega, 0 for the others)
   with the outer rule of `cfg` (Sec. 3, right-hand side (f, v)).  Entries
   of nodes that are not degrees of freedom are returned too.
   f_qp:     device [K][outer.n][n] values at the outer quadrature points, or
   f_affine: host [n][3], f_c(x) = f_affine[c][0] + f_affine[c][1] x_1
             + f_affine[c][2] x_2 (used when f_qp is NULL).
   Elements with a vertex index outside [0, M) are skipped (nlfem_build_pairs
   reports them as E_MESH; this call validates no device data).
   Allocates nothing and never synchronises.
   Errors: E_INVALID, E_HIP. */
int nlfem_rhs(const nlfem_mesh *mesh, const nlfem_config *cfg, const double *f_qp,
              const double *f_affine, double *b, void *stream);

/* Per-phase timing (diagnostic).  Bit p of `mask` enables phase p; 0 turns
   timing off.  While phase p is enabled, every call records a pair of HIP
   events on its stream around each launch group of that phase;
   nlfem_timing_read waits for them and returns the accumulated milliseconds
   and the number of timed groups per phase since the last reset.  Phases:
     0 geometry and grid     1 pair search        2 list sorting/linking
     3 CSR pattern           4 non-touching pair records (one kernel)
     5 touching pairs (one kernel)                6 row gather (one kernel)
     7 load vector           8 per-element sums of the non-touching
                               diagonal blocks (one kernel)
   nlfem_batch_assemble records its phases too (4, 5, 8, 6: one pair of
   events around the launches of each phase, the touching phase on the
   batch's second stream); replays of its HIP graph are not timed.
   Enabling creates events (host allocation); nlfem_assemble then still
   allocates no device memory.  Not thread-safe.
   Errors: E_INVALID (mask outside [0, 2^NLFEM_TIMING_PHASES)), E_HIP. */
#define NLFEM_TIMING_PHASES 9
int nlfem_timing_enable(int mask);
int nlfem_timing_read(double *ms, int64_t *launches, int reset);

/* Releases a handle and its device memory (synchronises the device). */
void nlfem_pairs_free(nlfem_pairs *pairs);

/* ------------------------------------------------------------------------
 * Batched assembly: many independent problems (meshes of uneven size, other
 * kernels, horizons and rules) in a few persistent launches over a global
 * work queue, one per phase and kernel specialisation, optionally replayed
 * from a HIP graph.  Results are bit-identical to nlfem_assemble of each
 * problem.  The paper assembles one problem at a time (Sec. 2.5, Alg. 1);
 * batching is a property of this implementation.
 * --------------------------------------------------------------------- */
typedef struct nlfem_batch nlfem_batch;   /* opaque, library-owned */
#define NLFEM_MAX_BATCH 4096

/* Fixes a batch of n problems: meshes[n], cfgs[n] (each as accepted by
   nlfem_assemble for pairs[i]; continuous ansatz only), pairs[n] (distinct built handles) and
   vals[n] (device output arrays, nnz of pairs[i] entries, owned by the
   caller).  All of them must stay valid and unchanged while the batch is
   used; the handles' workspaces are used by the batch.
   tune: 0 = default launch shapes; 1 = shapes from `tune_cache` (a text
   file, one line per device and batch structure) or, when absent, chosen by
   timing candidate shapes on this stream (per phase: queue shapes and one
   launch per problem) and appended to the file
   (tune_cache may be NULL: nothing is read or written); 2 = always timed.
   Tuning runs the assembly, so vals hold a valid result afterwards.
   Allocates device tables; synchronises.
   Errors: E_INVALID, E_MISMATCH, E_NOMEM, E_HIP, E_NODEVICE. */
int nlfem_batch_create(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs,
                       nlfem_pairs *const *pairs, double *const *vals, const char *tune_cache,
                       int32_t tune, nlfem_batch **batch, void *stream);

/* Assembles all problems of the batch into their vals on `stream`.
   Allocates nothing, records no memset (safe to capture into a HIP graph),
   and synchronises only to finish the check of a handle rebuilt without
   waiting (see nlfem_build_pairs).  Two runs of one batch must not overlap.
   Errors: E_INVALID, E_HIP, E_MISMATCH (a handle was built plainly since
   the batch was created), and the errors of a rebuild finished here. */
int nlfem_batch_assemble(nlfem_batch *batch, void *stream);

/* Same work from a HIP graph: the first call captures the launches of
   nlfem_batch_assemble on an internal stream and instantiates the graph
   (host allocation); every call launches it on `stream`.
   Errors: as nlfem_batch_assemble. */
int nlfem_batch_launch_graph(nlfem_batch *batch, void *stream);

/* Number of launch groups and the launch shape of the four phases
   (non-touching, touching, element diagonals, rows) as
   shape[8] = {chunk, workgroups per CU} x 4; {0, 0}: the phase runs as the
   single-problem launches of each problem in turn (the tuner's other
   candidate; same values).  Errors: E_INVALID. */
int nlfem_batch_info(const nlfem_batch *batch, int32_t *groups, int32_t *shape);

/* Releases a batch (synchronises the device).  NULL is ignored. */
void nlfem_batch_free(nlfem_batch *batch);

/* One-shot form: create (tune = 1 if tune_cache is given, else 0), assemble,
   synchronise, free.  Errors: those of nlfem_batch_create and _assemble. */
int nlfem_assemble_batched(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs,
                           nlfem_pairs *const *pairs, double *const *vals, const char *tune_cache,
                           void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
   harnesses that forbid hipMalloc): the one-shot batched assembly of
   nlfem_assemble_batched with its launch tables and work-queue counters in a
   static device array of NLFEM_NOALLOC_SCRATCH_BYTES (8 MiB) that each GPU
   the library runs on holds until the process ends.  Same arguments and
   results as nlfem_assemble_batched (default launch shapes, no tuning, no
   cache), all phases on `stream`.  Allocates no device memory (neither
   hipMalloc nor the nlfem_set_allocator hooks) and creates no stream or
   event; synchronises once, after copying the tables, then returns with the
   assembly enqueued.  Every call on one GPU shares that GPU's array, which
   keeps the last call's contents: calls that overlap in time on one GPU
   (from several host threads or streams) race and must not be made.
   Handles with an unchecked rebuild are rejected (E_INVALID; call
   nlfem_pairs_info first), since finishing one may need a plain build.
   Errors: those of nlfem_assemble_batched, and E_OVERFLOW when the batch's
   tables (about 7 KB per problem) exceed the array. */
#define NLFEM_NOALLOC_SCRATCH_BYTES (8u << 20)
int nlfem_assemble_batched_noalloc(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs,
                                   nlfem_pairs *const *pairs, double *const *vals, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NLFEM_H */
