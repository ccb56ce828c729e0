// Internal declarations of the gfx950 nonlocal assembler (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nlfem.h"

namespace nlfem {

constexpr int kMaxRule = 16;      // outer/inner rule points (2 status bits each in a u32)
constexpr int kMaxGauss = 32;     // 1-D Gauss points of the touching-pair rules
// Kernel specialisation flag: a weakly singular kernel (s <= 0) whose
// touching pairs take the standard rule with the ball (singular_n = 0), so
// point pairs at distance |z|^2 <= 1e-12 min(|det J_e|, |det J_f|) (the same
// point of both elements, up to rounding) are skipped (Sec. 2.4.2, Table 1:
// the rule that avoids x_p = y_q)
constexpr int kKerNoZeroDiv = 8;
inline int kernel_variant(const nlfem_config *c)
{
    return c->kernel != NLFEM_K_CONSTANT && c->singular_n == 0 ? c->kernel | kKerNoZeroDiv : c->kernel;
}
constexpr int kMaxPoly = 64;      // polygon vertices
constexpr int kWave = 64;

// status of one outer point with respect to an inner element
enum : uint32_t { kOut = 0u, kWhole = 1u, kStraddle = 2u };

// error bits raised by kernels, read back at synchronising calls
enum : int32_t {
    kErrIndex = 1,       // vertex index out of range
    kErrArea = 2,        // zero-area element
    kErrRowCap = 4,      // CSR row exceeded the symbolic capacity
    kErrSlot = 8,        // scatter target not in the pattern (internal bug)
    kErrCell = 16,       // cell occupancy above the pair-search tile size
    kErrClip = 32,       // polygon clip longer than the bound found by the pair search (internal bug)
    kErrEdge = 64,       // an edge shared by more than two elements (non-conforming mesh)
    kErrMaterial = 128,  // material id outside the configuration's table
};

// Material table of a label-dependent kernel: Psi(x, y) = c[m(x)][m(y)] Psi0
// (n = 0: no table, every coefficient 1).  Passed by value.
constexpr int kMaxMaterials = 4;
struct MatArgs {
    const int32_t *mat = nullptr;   // [K] material of each element
    int32_t n = 0;
    double c[kMaxMaterials * kMaxMaterials] = {};
    // coefficient of the ordered element pair (material of x's element first)
    __device__ double coef(int32_t ex, int32_t ey) const { return n == 0 ? 1.0 : c[mat[ex] * n + mat[ey]]; }
};
inline MatArgs material_args(const int32_t *mat, const nlfem_config *cfg)
{
    MatArgs m;
    if (cfg->n_materials > 0) {
        m.mat = mat;
        m.n = cfg->n_materials;
        for (int i = 0; i < m.n * m.n; ++i) m.c[i] = cfg->material_c[i];
    }
    return m;
}
// true when some c[a][b] != c[b][a]
inline bool material_nonsymmetric(const nlfem_config *cfg)
{
    const int n = cfg->n_materials;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < a; ++b)
            if (cfg->material_c[a * n + b] != cfg->material_c[b * n + a]) return true;
    return false;
}

// Quadrature tables passed by value (kernel arguments live in scalar registers).
struct RuleArgs {
    int32_t P, Q;
    int32_t same;                  // outer and inner rule identical
    double pxi[kMaxRule][2], pw[kMaxRule];
    double qxi[kMaxRule][2], qw[kMaxRule];
    double pphi[kMaxRule][3], qphi[kMaxRule][3];   // phi^ at the points
};

struct PolyArgs {
    int32_t N;
    double r_in;                   // inscribed radius (delta cos(pi/N) for the N-gon)
    double r_out;                  // largest distance of a polygon vertex from the centre
    double dir[kMaxPoly][2];
    double elen[kMaxPoly];         // delta |dir_{j+1} - dir_j|: edge lengths, for the margins of decisions
};

// the ball approaches clipped as polygons around each outer point: the
// inscribed N-gon and the infinity-norm square
// (and the paper's nocaps / approximate caps, whose polygons are built from
// the circle's crossings with the element instead: caps.h)
inline bool clipped_ball(int approach)
{
    return approach == NLFEM_A_APPROXCAPS_POLY || approach == NLFEM_A_INF_BALL || approach == NLFEM_A_NOCAPS ||
           approach == NLFEM_A_APPROXCAPS;
}

struct GaussArgs {
    int32_t n;
    double x[kMaxGauss], w[kMaxGauss];   // on [0, 1]
};

// Slots of the reduction buffer (u64 each), read back in one copy:
//   0-3 bounding-box keys, 4-5 radii, 6 candidate total, 7 elements of Omega
//   (discontinuous ansatz), 8 dof count, 9 longest
//   CSR row, 10 polygon clip bound, 11 CSR nnz, 12-17 totals of the
//   per-element pair counts, 18 error bits (int32), 19-24 largest
//   per-element pair counts (19: largest |S(e)|)
enum { kRedCounts = 6, kRedCand = 6, kRedDgDofs = 7, kRedDofs = 8, kRedMaxRow = 9, kRedClip = 10, kRedNnz = 11,
       kRedTot = 12, kRedErr = 18, kRedSegMax = 19, kRedSlots = 32 };

// Deep copy of a configuration (its host tables), for a build that may have
// to run again after the call that gave it has returned.
struct ConfigCopy {
    nlfem_config c{};
    std::vector<double> oxi, ow, ixi, iw, dirs;
    void set(const nlfem_config &src)
    {
        c = src;
        oxi.assign(src.outer.xi, src.outer.xi + 2 * src.outer.n);
        ow.assign(src.outer.w, src.outer.w + src.outer.n);
        ixi.assign(src.inner.xi, src.inner.xi + 2 * src.inner.n);
        iw.assign(src.inner.w, src.inner.w + src.inner.n);
        if (src.polygon_dirs && src.polygon_n > 0) dirs.assign(src.polygon_dirs, src.polygon_dirs + 2 * src.polygon_n);
        else dirs.clear();
        c.outer.xi = oxi.data();
        c.outer.w = ow.data();
        c.inner.xi = ixi.data();
        c.inner.w = iw.data();
        c.polygon_dirs = dirs.empty() ? nullptr : dirs.data();
    }
};

// A block of device memory and the allocator that gave it (nlfem_set_allocator:
// the caller's hook, else hipMalloc/hipFree).  abi.hip.
struct DevBlock {
    void *p = nullptr;
    size_t cap = 0;
    nlfem_free_fn free_fn = nullptr;   // null: hipFree
    void *ctx = nullptr;
    hipStream_t stream = nullptr;      // stream of the allocation
};
// allocates `bytes` (256-byte aligned) on stream s into b (b must be empty)
int dev_alloc(DevBlock &b, size_t bytes, hipStream_t s);
// releases b (work already enqueued on its stream may still use it when the
// hook is stream-ordered; hipFree waits for the device)
void dev_release(DevBlock &b);

// A rebuild launched with the last build's sizes: a build kernel runs only
// while the reduction slots that are final at its launch (mask) equal the
// last build's (want, on the device); the error slot is among them.
struct SpecGate {
    const unsigned long long *red = nullptr;    // nullptr: not gated
    const unsigned long long *want = nullptr;   // [kRedSlots]
    uint32_t mask = 0;
};

// true when a compared slot differs: the calling wave returns.  Every lane of
// the wave calls it, and every wave of a workgroup gets the same answer.
__device__ inline bool gated(const SpecGate &g)
{
    if (!g.red) return false;
    const int lane = threadIdx.x & 63;
    bool bad = false;
    if (lane < kRedSlots && ((g.mask >> lane) & 1u)) bad = g.red[lane] != g.want[lane];
    return __any(bad);
}

// up to kZeroMax ranges of 32-bit words cleared by one launch
constexpr int kZeroMax = 12;
struct ZeroList {
    uint32_t *p[kZeroMax];
    int64_t n[kZeroMax];
    int cnt;
    template <class T>
    void add(T *ptr, int64_t count)   // count elements of T (a multiple of 4 bytes)
    {
        static_assert(sizeof(T) % 4 == 0, "32-bit words");
        p[cnt] = (uint32_t *)ptr;
        n[cnt] = count * (int64_t)(sizeof(T) / 4);
        ++cnt;
    }
};

// workspace of one chained scan of up to `tiles` tiles: hdr = [1 + tiles]
// (ticket, per-tile words), zero before the launch
struct ScanWork {
    int64_t *hdr = nullptr;
    int64_t tiles = 0;
};

// counters filled by the pair search (ordered pairs per class)
enum { kCntPairs = 0, kCntFar, kCntVertex, kCntEdge, kCntIdent, kCntLast };

// per-element count arrays of the pair search, each [K + 1]
enum { kLsS = 0, kLsP, kLsUF, kLsUI, kLsUE, kLsUV, kLsLast };

}  // namespace nlfem

struct nlfem_pairs {
    int device = 0;
    // what the handle was built from
    const double *mesh_vertices = nullptr;
    const int32_t *mesh_elements = nullptr;
    const int32_t *mesh_labels = nullptr;
    const int32_t *mesh_materials = nullptr;   // validated by the build when a table is given
    int64_t M = 0, K = 0;
    int32_t ncomp = 1;
    int32_t kernel = 0, approach = 0, singular = 0;
    int32_t dg = 0;              // discontinuous ansatz
    // material table given at build / non-symmetric: edge and vertex touching
    // pairs then take the 4D transforms over the pair's six element unknowns
    // (the records of the discontinuous path), scaled per column in the rows
    int32_t materials = 0, nonsym = 0;
    double delta = 0.0;
    nlfem::RuleArgs rules{};
    nlfem::PolyArgs poly{};
    // counts
    int64_t nS = 0, nP = 0, nUF = 0, nUT = 0, nUTc[3] = {0, 0, 0};   // ident, edge, vertex
    int64_t n_pairs = 0, n_far = 0, n_vertex = 0, n_edge = 0, n_ident = 0;
    int64_t n_dof = 0, nnz_node = 0;
    int32_t hcap = 0;
    // grid
    double gx0 = 0, gy0 = 0, gh = 0, far_reach = 0;
    int64_t max_S = 0;
    int32_t gnx = 0, gny = 0, gr = 2;   // gr: neighbour-cell radius
    int32_t max_clip = 0;        // largest intermediate vertex count of a straddling polygon clip
    // ---- device memory (grow-only buffers, sized by cap_*) ----
    // element geometry (SoA)
    double2 *v0 = nullptr;       // [K]
    double4 *J = nullptr;        // [K]  (J00, J01, J10, J11), J = [v1 - v0, v2 - v0]
    double *det = nullptr;       // [K]  |det J|
    double2 *bary = nullptr;     // [K]
    double2 *xp = nullptr;       // [K * P] outer quadrature points (FP64)
    uint32_t *node_flags = nullptr;  // [M] bit0 vertex of an Omega element, bit1 of an Omega_D one
    int32_t *err = nullptr;      // [1] error bits
    unsigned long long *red = nullptr;   // [kRedSlots] reduction slots (see kRed*)
    unsigned long long *rb = nullptr;    // [kRedSlots] pinned host copy of red
    // rebuilds with the sizes of the last build: expected reduction slots and
    // the gate the build kernels test while such a build runs
    bool spec_ok = false;
    unsigned long long spec_red[nlfem::kRedSlots] = {};   // host copy
    unsigned long long *spec_want = nullptr;              // device copy
    nlfem::SpecGate gate{};
    // a rebuild whose read-back has not been checked yet: what a plain build
    // needs if the check fails, and the gate of assembly launches until then
    bool pending = false;
    nlfem_mesh pend_mesh{};
    nlfem::ConfigCopy pend_cfg;
    hipStream_t pend_stream = nullptr;
    nlfem::SpecGate asm_gate{};
    uint64_t generation = 0;   // counts plain builds (batches check it)
    int32_t last_build = 0;   // 0 plain, 1 speculative rebuild held, 2 it fell back
    unsigned long long *counters = nullptr;  // [kCntLast]
    // node -> element incidence
    int64_t *ne_ptr = nullptr;   // [M + 1]
    int32_t *ne_list = nullptr;  // [3K]
    int32_t *ne_fill = nullptr;  // [M]
    // grid
    int64_t *cell_cnt = nullptr;    // [ncell + 1]
    int64_t *cell_start = nullptr;  // [ncell + 1]
    int32_t *cell_fill = nullptr;   // [ncell]
    int32_t *cell_elems = nullptr;  // [K]
    int32_t *cell_of = nullptr;     // [K]
    // per-element counts and offsets [kLsLast][K + 1]
    int64_t *lcnt = nullptr;
    int64_t *loff = nullptr;
    int64_t *scan_tmp = nullptr;   // the workspaces of the build's four scans
    nlfem::ScanWork scan_w[4];     // node/cell/code buckets, candidates, list counts, row lengths
    int64_t scan_hdr = 0;          // their words
    // symmetric neighbour list S(e) = {f : (e,f) or (f,e) interacts}, each
    // segment sorted by neighbour id
    int32_t *snbr = nullptr;     // [nS]
    uint8_t *sflag = nullptr;    // [nS] bit0 (e,f) in P, bit1 (f,e) in P, bits 2-3 class
    int32_t *srec = nullptr;     // [nS] record of the unordered pair (far or touching list)
    int4 *snode = nullptr;       // [nS] (f, the three vertices of f): one load for the row kernels
    // unsorted lists written by the pair search, element e's in the segment
    // [scr_off[e], scr_off[e] + |S(e)|) of a scratch sized by the candidates
    // the search visits (cand[e])
    int64_t *cand = nullptr;     // [K]
    int64_t *scr_off = nullptr;  // [K + 1]
    int64_t total_cand = 0;
    int32_t *snbr_tmp = nullptr;
    uint8_t *sflag_tmp = nullptr;
    uint2 *smask_tmp = nullptr;
    // unordered non-touching pairs e <= f (far work list)
    int32_t *ue = nullptr, *uf = nullptr;     // [nUF]
    uint2 *um = nullptr;
    // unordered touching pairs e <= f: [ident | edge | vertex]
    int32_t *te = nullptr, *tf = nullptr;     // [nUT]
    // degree-of-freedom nodes (the rows of the matrix) in the Morton order of
    // their grid cells, so that rows worked on together are close in space
    int32_t *dof_list = nullptr; // [M], first n_dof entries used
    int32_t morton_bits = 0;     // bits per axis of the cell codes
    int32_t *node_code = nullptr;        // [M] cell code of a dof node, -1 otherwise
    int64_t *code_cnt = nullptr;         // [ncode + 1] dof nodes per code
    int64_t *code_start = nullptr;       // [ncode + 1]
    int32_t *code_fill = nullptr;        // [ncode]
    // node-level CSR of degree-of-freedom rows
    int64_t *nlen = nullptr;     // [M + 1]
    int64_t *nptr = nullptr;     // [M + 1]
    int32_t *ncol = nullptr;     // [nnz_node]
    int32_t *csr_stage = nullptr;   // [n_dof][csr_slot(hcap)] sorted rows before packing
    int64_t max_row = 0;         // longest node row
    // per-pair results of the assembly (workspace held by the handle)
    void *far_rec = nullptr;     // nUF records of far_stride values (layout by use: row chunks, column chunks, diagonal blocks), FP32 (mixed) or FP64
    double *touch_rec = nullptr; // [nUT][touch_stride]
    double *dsum = nullptr;      // [K][6 * NK] summed element-diagonal blocks of the far pairs
    double *poly_dir = nullptr;  // [N][2] polygon directions (approach POLY)
    int32_t far_stride = 0, touch_stride = 0;
    // discontinuous ansatz: element blocks of each row block and their prefix
    int64_t *dg_cnt = nullptr;   // [K]
    int64_t *dg_ptr = nullptr;   // [K + 1]
    hipEvent_t ev_rb = nullptr;    // completion of a read-back of the reduction slots
    // assemblies queued while a rebuild was unchecked, and those of them
    // whose work was skipped because the rebuild found other sizes
    int64_t pend_asm = 0, skipped = 0;
    hipStream_t alloc_stream = nullptr;   // stream of the build that allocates
    // grow-only device buffers behind the typed pointers above
    nlfem::DevBlock bufs[64];
};

namespace nlfem {

// per-phase timing (abi.hip): no-ops unless enabled ------------------------
enum { kPhGeometry = 0, kPhPairs, kPhLists, kPhCsr, kPhFar, kPhTouch, kPhRows, kPhRhs, kPhDiag, kPhLast };
void timing_begin(int phase, hipStream_t s);
void timing_end(int phase, hipStream_t s);

// error reporting (abi.hip) --------------------------------------------
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
// abi.hip: finishes an unchecked rebuild of h (waits for its read-back; runs
// the plain build when the sizes differ)
int resolve(nlfem_pairs *h);

#define NLFEM_HIP(call)                                               \
    do {                                                              \
        hipError_t _e = (call);                                       \
        if (_e != hipSuccess) return ::nlfem::hip_error(_e, #call);   \
    } while (0)

// rows of the row kernels per workgroup: one wave each, synchronised per wave
constexpr int kWavesPerRowBlock = 4;

// makes the LDS writes of the wave's lanes visible to its other lanes
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define NLFEM_TRY(x)                     \
    do {                                 \
        int _rc = (x);                   \
        if (_rc != NLFEM_OK) return _rc; \
    } while (0)

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b % 8) and every XCD has its own L2.  Kernels whose neighbouring items
// (node rows, elements) read the same records let block b take item
// (b % 8) * per + b / 8, per = ceil(n / 8), so that each XCD walks one
// contiguous range of items.  Grids are multiples of 8 (xcd_grid) and
// grid-stride loops step by gridDim.x, which keeps b % 8.
constexpr int kXcd = 8;
inline unsigned xcd_grid(int64_t n, int64_t cap = 1 << 20)
{
    const int64_t g = kXcd * ((n + kXcd - 1) / kXcd);
    return (unsigned)(g < cap ? g : cap);
}
__device__ inline int64_t xcd_span(int64_t n) { return kXcd * ((n + kXcd - 1) / kXcd); }
__device__ inline int64_t xcd_item(int64_t b, int64_t n)
{
    const int64_t per = (n + kXcd - 1) / kXcd;
    return (b % kXcd) * per + b / kXcd;
}

// scan.hip: out[0..n] = exclusive prefix sums of in[0..n-1], out[n] = total
// (also written to *total when given; device pointer).  n = 0 gives out[0] = 0.
// *maxval (device, zero before the call) receives the largest input when
// given.  One launch; the workspace must be zero when the launch starts.
int exclusive_scan(const int64_t *in, int64_t *out, int64_t n, const ScanWork &w, hipStream_t s,
                   int64_t *total = nullptr, int64_t *maxval = nullptr, const SpecGate &gate = SpecGate{});
// the same for nseg segments of `stride` slots (segment k at in + k * stride),
// totals[k] = total and maxes[k] = largest input of segment k when given
int exclusive_scan_segments(const int64_t *in, int64_t *out, int64_t n, int nseg, int64_t stride,
                            const ScanWork &w, int64_t *totals, hipStream_t s, int64_t *maxes = nullptr,
                            const SpecGate &gate = SpecGate{});
// up to kScanParts independent arrays in one launch; the workspace needs the
// sum of scan_tiles(n_k) over the parts
constexpr int kScanParts = 8;
struct ScanPart {
    const int64_t *in;
    int64_t *out;       // [n + 1]
    int64_t n;
    int64_t *total;     // device, optional
    int64_t *maxv;      // device, optional
};
int exclusive_scan_multi(const ScanPart *parts, int cnt, const ScanWork &w, hipStream_t s,
                         const SpecGate &gate = SpecGate{});
// tiles of a scan of nseg arrays of n counts
int64_t scan_tiles(int64_t n, int nseg = 1);
double key_to_double(unsigned long long key);

// geometry.hip
// also clears the ranges of `later` in its first launch
int launch_geometry(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s, const ZeroList &later);
int launch_zero(const ZeroList &z, unsigned long long *init_red, hipStream_t s);
// grid + pairs (pairs.hip)
// node -> element incidence counts (nlen), grid cell counts (cell_cnt) and
// dof nodes per cell code (code_cnt; their scan total is the dof count)
int launch_bucket_count(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s);
// incidence lists, cell element lists and the dof-node list in code order
// (needs ne_ptr, cell_start and code_start); clears nlen
int launch_bucket_fill(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s);
// one pass: the neighbour entries of every element into its scratch segment
// (scr_off), the six per-element counts into lcnt
int launch_pairs(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s);
// lists.hip: sorted neighbour lists, work lists and record links
int launch_sort_lists(nlfem_pairs *h, hipStream_t s);
// csr.hip
// staged rows: one slot of csr_slot(hcap) ids per dof row
inline int32_t csr_slot(int32_t hcap) { return hcap / 4 * 3; }
// -> nlen, stage, max row; with links also the mirror records of the lower
// neighbour-list entries (after the list sort)
int launch_csr_rows(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s, bool links, bool rows = true);
// stage -> ncol; with slots_out (pinned host) also copies the reduction slots
int launch_csr_pack(nlfem_pairs *h, hipStream_t s, unsigned long long *slots_out = nullptr);
int launch_pattern(const nlfem_pairs *h, int64_t *row_ptr, int32_t *col, hipStream_t s);
int launch_export(const nlfem_pairs *h, int32_t *k, int32_t *l, int8_t *cls, hipStream_t s);
// assemble.hip
int far_record_stride(int ncomp);     // values per non-touching pair record
int touch_record_stride(int ncomp, bool dg);   // values per touching pair record
// dg.hip: discontinuous ansatz
int launch_dg_counts(nlfem_pairs *h, hipStream_t s);
int launch_dg_pattern(const nlfem_pairs *h, int64_t *row_ptr, int32_t *col, hipStream_t s);
int launch_dg_assemble_rest(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, const GaussArgs &g,
                            double *val, hipStream_t s);
int launch_dg_rows(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg, double *val, hipStream_t s);
int launch_assemble(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *cfg,
                    const GaussArgs &g, double *val, hipStream_t s);
// rhs.hip
int launch_rhs(const nlfem_mesh *m, const RuleArgs &r, int ncomp, const double *f_qp,
               const double *f_affine, double *b, hipStream_t s, bool dg = false);

}  // namespace nlfem
