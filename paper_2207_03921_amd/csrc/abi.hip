// Exported C ABI: argument validation, handle life cycle, device buffers and
// the order of the build steps.  All arithmetic happens in the kernels of the
// other translation units.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "batch.h"
#include "nlfem_internal.h"

namespace nlfem {

namespace {
thread_local std::string g_err = "no error";

// device allocator (nlfem_set_allocator) and the capacity limit of a build
struct Allocator {
    nlfem_alloc_fn alloc = nullptr;
    nlfem_free_fn free_fn = nullptr;
    void *ctx = nullptr;
};
Allocator g_alloc;
int64_t g_capacity = 0;

enum Buf : int {
    B_V0, B_J, B_DET, B_BARY, B_XP, B_FLAGS, B_ERR, B_RED, B_NEPTR, B_NELIST, B_NEFILL,
    B_CELLCNT, B_CELLSTART, B_CELLFILL, B_CELLELEMS, B_CELLOF, B_LCNT, B_LOFF, B_SCAN,
    B_SNBR, B_SFLAG, B_SREC, B_SNBRT, B_SFLAGT, B_SMASKT, B_UE, B_UF, B_UM, B_TE, B_TF,
    B_NLEN, B_NPTR, B_NCOL, B_FARREC, B_TOUCHREC, B_DSUM, B_DOFL, B_POLYDIR, B_CSRSTAGE, B_SNODE, B_SPEC,
    B_NCODE, B_CODECNT, B_CODESTART, B_CODEFILL, B_CAND, B_SCROFF, B_DGCNT, B_DGPTR, B_LAST
};
static_assert(B_LAST <= (int)(sizeof(nlfem_pairs::bufs) / sizeof(nlfem_pairs::bufs[0])), "too few buffer slots");


int ensure(nlfem_pairs *h, int id, size_t bytes)
{
    auto &b = h->bufs[id];
    if (bytes == 0) bytes = 16;
    if (b.p && b.cap >= bytes) return NLFEM_OK;
    if (b.p) dev_release(b);
    return dev_alloc(b, bytes + bytes / 8, h->alloc_stream);   // headroom for rebuilds that grow a little
}

template <typename T>
int ensure_typed(nlfem_pairs *h, int id, int64_t n, T *&ptr)
{
    int rc = ensure(h, id, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    if (rc) return rc;
    ptr = (T *)h->bufs[id].p;
    return NLFEM_OK;
}


// Gauss-Legendre nodes and weights on [0, 1]: Newton's method on P_n, with P_n
// from the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;   // P_0, P_1
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);   // P_n'(z)
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - z);   // z descends with i, so x ascends on [0, 1]
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

bool is_finite(double v) { return std::isfinite(v); }

int check_rule(const nlfem_rule &r, const char *which)
{
    if (r.n < 1 || r.n > kMaxRule)
        return set_error(NLFEM_E_INVALID, std::string(which) + " rule: n must be in [1, 16]");
    if (!r.xi || !r.w) return set_error(NLFEM_E_INVALID, std::string(which) + " rule: NULL table");
    double s = 0.0;
    for (int p = 0; p < r.n; ++p) {
        if (!is_finite(r.xi[2 * p]) || !is_finite(r.xi[2 * p + 1]) || !is_finite(r.w[p]))
            return set_error(NLFEM_E_INVALID, std::string(which) + " rule: non-finite entry");
        s += r.w[p];
    }
    if (std::fabs(s - 0.5) > 1e-12)
        return set_error(NLFEM_E_INVALID, std::string(which) + " rule: weights must sum to 1/2");
    return NLFEM_OK;
}

int check_mesh(const nlfem_mesh *m)
{
    if (!m) return set_error(NLFEM_E_INVALID, "mesh is NULL");
    if (m->n_vertices < 1 || m->n_elements < 1)
        return set_error(NLFEM_E_INVALID, "mesh needs at least one vertex and one element");
    if (m->n_vertices > (int64_t)INT32_MAX / 2 || m->n_elements > (int64_t)INT32_MAX / 4)
        return set_error(NLFEM_E_OVERFLOW, "mesh too large for 32-bit indices");
    if (!m->vertices || !m->elements || !m->labels) return set_error(NLFEM_E_INVALID, "mesh array is NULL");
    return NLFEM_OK;
}

int check_cfg(const nlfem_config *c)
{
    if (!c) return set_error(NLFEM_E_INVALID, "config is NULL");
    if (c->kernel < NLFEM_K_CONSTANT || c->kernel > NLFEM_K_FRAC_HALF)
        return set_error(NLFEM_E_INVALID, "unknown kernel");
    if (!is_finite(c->c)) return set_error(NLFEM_E_INVALID, "kernel constant must be finite");
    if (!(c->delta > 0.0) || !is_finite(c->delta)) return set_error(NLFEM_E_INVALID, "delta must be positive");
    if (c->approach < NLFEM_A_NOCAPS_BARY || c->approach > NLFEM_A_APPROXCAPS)
        return set_error(NLFEM_E_INVALID, "unknown ball approach");
    if (c->precision != NLFEM_P_FP64 && c->precision != NLFEM_P_MIXED)
        return set_error(NLFEM_E_INVALID, "unknown precision");
    if (c->singular_n < 0 || c->singular_n > kMaxGauss)
        return set_error(NLFEM_E_INVALID, "singular_n must be in [0, 32]");
    if (c->ansatz != NLFEM_ANSATZ_CG && c->ansatz != NLFEM_ANSATZ_DG)
        return set_error(NLFEM_E_INVALID, "unknown ansatz");
    if (c->kernel == NLFEM_K_FRAC_HALF && c->singular_n == 0)
        return set_error(NLFEM_E_INVALID,
                         "the s = 1/2 kernel needs singular_n > 0 (regularising transforms on touching pairs)");
    NLFEM_TRY(check_rule(c->outer, "outer"));
    NLFEM_TRY(check_rule(c->inner, "inner"));
    if (c->n_materials < 0 || c->n_materials > kMaxMaterials)
        return set_error(NLFEM_E_INVALID, "n_materials must be in [0, 4]");
    if (c->n_materials > 0) {
        if (!c->material_c) return set_error(NLFEM_E_INVALID, "material_c is NULL");
        for (int i = 0; i < c->n_materials * c->n_materials; ++i)
            if (!is_finite(c->material_c[i])) return set_error(NLFEM_E_INVALID, "material_c not finite");
        if (c->kernel == NLFEM_K_FRAC_HALF && material_nonsymmetric(c))
            return set_error(NLFEM_E_INVALID,
                             "a non-symmetric material table needs a kernel with s <= 0 (not the s = 1/2 kernel)");
    }
    if (c->approach == NLFEM_A_APPROXCAPS_POLY) {
        if (c->polygon_n < 3 || c->polygon_n > kMaxPoly)
            return set_error(NLFEM_E_INVALID, "polygon_n must be in [3, 64]");
        if (!c->polygon_dirs) return set_error(NLFEM_E_INVALID, "polygon_dirs is NULL");
        const int N = c->polygon_n;
        for (int j = 0; j < N; ++j) {
            const double *a = c->polygon_dirs + 2 * j, *b = c->polygon_dirs + 2 * ((j + 1) % N);
            const double *d = c->polygon_dirs + 2 * ((j + 2) % N);
            if (!is_finite(a[0]) || !is_finite(a[1])) return set_error(NLFEM_E_INVALID, "polygon_dirs not finite");
            // convex, counter-clockwise and containing the centre
            if ((b[0] - a[0]) * (d[1] - b[1]) - (b[1] - a[1]) * (d[0] - b[0]) <= 0.0 ||
                a[0] * b[1] - a[1] * b[0] <= 0.0)
                return set_error(NLFEM_E_INVALID, "polygon must be convex, counter-clockwise, around 0");
        }
    }
    return NLFEM_OK;
}

RuleArgs make_rules(const nlfem_config *c)
{
    RuleArgs r{};
    r.P = c->outer.n;
    r.Q = c->inner.n;
    for (int p = 0; p < r.P; ++p) {
        r.pxi[p][0] = c->outer.xi[2 * p];
        r.pxi[p][1] = c->outer.xi[2 * p + 1];
        r.pw[p] = c->outer.w[p];
        r.pphi[p][0] = 1.0 - r.pxi[p][0] - r.pxi[p][1];
        r.pphi[p][1] = r.pxi[p][0];
        r.pphi[p][2] = r.pxi[p][1];
    }
    for (int q = 0; q < r.Q; ++q) {
        r.qxi[q][0] = c->inner.xi[2 * q];
        r.qxi[q][1] = c->inner.xi[2 * q + 1];
        r.qw[q] = c->inner.w[q];
        r.qphi[q][0] = 1.0 - r.qxi[q][0] - r.qxi[q][1];
        r.qphi[q][1] = r.qxi[q][0];
        r.qphi[q][2] = r.qxi[q][1];
    }
    r.same = r.P == r.Q && std::memcmp(r.pxi, r.qxi, sizeof(double) * 2 * r.P) == 0 &&
             std::memcmp(r.pw, r.qw, sizeof(double) * r.P) == 0;
    return r;
}

PolyArgs make_poly(const nlfem_config *c)
{
    PolyArgs p{};
    if (!clipped_ball(c->approach)) return p;
    if (c->approach == NLFEM_A_NOCAPS || c->approach == NLFEM_A_APPROXCAPS) {
        // polygons inside the disc, built from its crossings with the element
        p.N = 0;
        p.r_in = p.r_out = c->delta;
        return p;
    }
    if (c->approach == NLFEM_A_INF_BALL) {
        // Def. 2.5: corners x + delta (+-1, +-1), counter-clockwise from (+1, +1)
        static const double sq[4][2] = {{1.0, 1.0}, {-1.0, 1.0}, {-1.0, -1.0}, {1.0, -1.0}};
        p.N = 4;
        std::memcpy(p.dir, sq, sizeof sq);
    } else {
        p.N = c->polygon_n;
        for (int j = 0; j < p.N; ++j) {
            p.dir[j][0] = c->polygon_dirs[2 * j];
            p.dir[j][1] = c->polygon_dirs[2 * j + 1];
        }
    }
    double rmin = 1e300, rmax = 0.0;
    for (int j = 0; j < p.N; ++j) {
        const int j1 = (j + 1) % p.N;
        const double ex = p.dir[j1][0] - p.dir[j][0], ey = p.dir[j1][1] - p.dir[j][1];
        const double cr = p.dir[j][0] * p.dir[j1][1] - p.dir[j][1] * p.dir[j1][0];
        rmin = std::min(rmin, cr / std::sqrt(ex * ex + ey * ey));
        rmax = std::max(rmax, std::sqrt(p.dir[j][0] * p.dir[j][0] + p.dir[j][1] * p.dir[j][1]));
        p.elen[j] = c->delta * std::sqrt(ex * ex + ey * ey);
    }
    p.r_in = c->delta * rmin;
    p.r_out = c->delta * rmax;
    return p;
}

int ncomp_of(int kernel) { return kernel == NLFEM_K_PERIDYNAMIC ? 2 : 1; }

int check_device()
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return set_error(NLFEM_E_NODEVICE, "no HIP device available");
    }
    return NLFEM_OK;
}

// Slots a speculative rebuild compares with the last build's, by the point
// of the build where they are final: after the geometry (bounding box, radii,
// error bits), after the pair search (dofs, clip bound, list totals and
// maxima), after the symbolic pass (longest row, nnz).
constexpr uint32_t kSpecGeo = 0x3fu | (1u << kRedErr);
constexpr uint32_t kSpecCand = kSpecGeo | (1u << kRedCand);   // the search's scratch size
constexpr uint32_t kSpecPairs =
    kSpecCand | (1u << kRedDofs) | (1u << kRedClip) | (0x3fu << kRedTot) | (0x3fu << kRedSegMax);
constexpr uint32_t kSpecCsr = kSpecPairs | (1u << kRedMaxRow) | (1u << kRedNnz);

// Copies the reduction slots to the pinned host buffer and waits for them.
// The wait polls an event rather than blocking in the runtime: it lasts tens
// of microseconds, and a blocking wait adds the wake-up of the host thread.
int wait_event(hipEvent_t ev)
{
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return NLFEM_OK;
        if (e != hipErrorNotReady) return hip_error(e, "hipEventQuery");
    }
}

int read_slots(nlfem_pairs *h, hipStream_t s)
{
    NLFEM_HIP(hipMemcpyAsync(h->rb, h->red, sizeof(unsigned long long) * kRedSlots, hipMemcpyDeviceToHost, s));
    NLFEM_HIP(hipEventRecord(h->ev_rb, s));
    return wait_event(h->ev_rb);
}

// true when the read-back of a rebuild (pinned copy) has the slots of the
// last plain build
bool rebuild_held(const nlfem_pairs *h)
{
    for (int i = 0; i < kRedSlots; ++i)
        if (((kSpecCsr >> i) & 1u) && h->rb[i] != h->spec_red[i]) return false;
    return true;
}

// Counters of the build after the geometry, all cleared by one launch.
// codes of the order of the dof rows: the Morton codes of the grid cells
// (2 * bits interleaved bits), or the row-major cell index for grids too
// elongated for a compact Morton range (morton_bits < 0)
int64_t morton_codes(const nlfem_pairs *h)
{
    return h->morton_bits >= 0 ? (int64_t)1 << (2 * h->morton_bits) : (int64_t)h->gnx * h->gny;
}

ZeroList build_counters(nlfem_pairs *h)
{
    const int64_t ncell = (int64_t)h->gnx * h->gny;
    ZeroList z{};
    z.add(h->cell_cnt, ncell + 1);
    z.add(h->cell_fill, ncell);
    z.add(h->code_cnt, morton_codes(h) + 1);
    z.add(h->code_fill, morton_codes(h));
    z.add(h->lcnt, kLsLast * (h->K + 1));
    z.add(h->nlen, h->M + 1);
    z.add(h->ne_fill, h->M);
    z.add(h->scan_tmp, h->scan_hdr);   // tickets and flags of the chained scans
    return z;
}

// Rest of a plain build for the discontinuous ansatz, after the lists: the
// mirror links, the element blocks of every row block and their prefix sums
// (the pattern follows from the sorted lists, so there is no symbolic pass),
// and the assembly's workspace.
int build_dg_rest(nlfem_pairs *h, const nlfem_mesh *m, hipStream_t s)
{
    const int64_t K = h->K;
    unsigned long long *red = h->rb;
    NLFEM_TRY(ensure_typed(h, B_DGCNT, K, h->dg_cnt));
    NLFEM_TRY(ensure_typed(h, B_DGPTR, K + 1, h->dg_ptr));
    timing_begin(kPhCsr, s);
    NLFEM_TRY(launch_csr_rows(h, m, s, true, false));
    NLFEM_TRY(launch_dg_counts(h, s));
    NLFEM_TRY(exclusive_scan(h->dg_cnt, h->dg_ptr, K, h->scan_w[3], s, (int64_t *)(h->red + kRedNnz),
                             (int64_t *)(h->red + kRedMaxRow), h->gate));
    timing_end(kPhCsr, s);
    NLFEM_TRY(read_slots(h, s));
    const int32_t err = (int32_t)(red[kRedErr] & 0xffffffffull);
    if (err & kErrEdge) return set_error(NLFEM_E_MESH, "an edge is shared by more than two elements");
    if (err) return set_error(NLFEM_E_OVERFLOW, "internal capacity exceeded during the pair search");
    const int64_t blocks = (int64_t)red[kRedNnz];
    if (9 * blocks * h->ncomp * h->ncomp >= (int64_t)INT32_MAX * 64)
        return set_error(NLFEM_E_OVERFLOW, "matrix too large");
    h->nnz_node = 9 * blocks;   // nnz = nnz_node * n^2
    h->n_dof = 3 * (int64_t)red[kRedDgDofs];
    h->max_row = 3 * (int64_t)red[kRedMaxRow];
    h->far_stride = far_record_stride(h->ncomp);
    h->touch_stride = touch_record_stride(h->ncomp, true);
    double *far_rec = nullptr;
    NLFEM_TRY(ensure_typed(h, B_FARREC, h->nUF * h->far_stride, far_rec));
    h->far_rec = far_rec;
    NLFEM_TRY(ensure_typed(h, B_TOUCHREC, h->nUT * h->touch_stride, h->touch_rec));
    NLFEM_TRY(ensure_typed(h, B_DSUM, K * 6 * (h->ncomp == 1 ? 1 : 3), h->dsum));
    h->spec_ok = false;   // rebuilds of the discontinuous ansatz are plain builds
    ++h->generation;
    return NLFEM_OK;
}

// Builds the pair structures.  The plain build reads the reduction slots
// back three times to size buffers and launches.  A speculative rebuild
// (spec: same sizes and configuration as the handle's last build) launches
// everything with the last build's sizes, and every build kernel after the
// geometry first compares the slots final by its launch with the last
// build's (on the device) and returns when one differs.  Its read-back is
// checked by the next call that uses the handle (resolve), which runs the
// plain build when a slot differs.
int build(const nlfem_mesh *m, const nlfem_config *cfg, nlfem_pairs *h, hipStream_t s, bool spec)
{
    h->gate = SpecGate{};
    if (!spec) h->spec_ok = false;
    h->alloc_stream = s;
    NLFEM_HIP(hipGetDevice(&h->device));
    h->mesh_vertices = m->vertices;
    h->mesh_elements = m->elements;
    h->mesh_labels = m->labels;
    h->M = m->n_vertices;
    h->K = m->n_elements;
    h->kernel = cfg->kernel;
    h->ncomp = ncomp_of(cfg->kernel);
    h->approach = cfg->approach;
    h->singular = cfg->singular_n > 0;
    h->dg = cfg->ansatz == NLFEM_ANSATZ_DG;
    h->materials = cfg->n_materials;
    h->mesh_materials = cfg->n_materials > 0 ? m->materials : nullptr;
    h->nonsym = cfg->n_materials > 0 && material_nonsymmetric(cfg);
    h->delta = cfg->delta;
    h->rules = make_rules(cfg);
    h->poly = make_poly(cfg);
    const int64_t K = h->K, M = h->M, K1 = K + 1, P = h->rules.P;

    // geometry ---------------------------------------------------------
    NLFEM_TRY(ensure_typed(h, B_V0, K, h->v0));
    NLFEM_TRY(ensure_typed(h, B_J, K, h->J));
    NLFEM_TRY(ensure_typed(h, B_DET, K, h->det));
    NLFEM_TRY(ensure_typed(h, B_BARY, K, h->bary));
    NLFEM_TRY(ensure_typed(h, B_XP, K * P, h->xp));
    NLFEM_TRY(ensure_typed(h, B_FLAGS, M, h->node_flags));
    NLFEM_TRY(ensure_typed(h, B_RED, kRedSlots, h->red));
    h->err = (int32_t *)(h->red + kRedErr);
    if (!h->rb) {
        void *rb = nullptr;
        // coherent: a kernel of a rebuild writes the slots here directly
        NLFEM_HIP(hipHostMalloc(&rb, sizeof(unsigned long long) * kRedSlots, hipHostMallocCoherent));
        h->rb = (unsigned long long *)rb;
    }
    unsigned long long *red = h->rb;
    if (!h->ev_rb) {
        NLFEM_HIP(hipEventCreateWithFlags(&h->ev_rb, hipEventDisableTiming));
    }
    timing_begin(kPhGeometry, s);
    {
        // a rebuild clears the later counters (last build's sizes) here too
        const ZeroList later = spec ? build_counters(h) : ZeroList{};
        NLFEM_TRY(launch_geometry(h, m, s, later));
    }
    timing_end(kPhGeometry, s);
    int32_t err = 0;
    if (spec) {
        // the grid of the last build holds while the box and radii are equal
        h->gate = SpecGate{h->red, h->spec_want, kSpecGeo};
    } else {
        NLFEM_TRY(read_slots(h, s));
        err = (int32_t)(red[kRedErr] & 0xffffffffull);
        if (err & kErrIndex) return set_error(NLFEM_E_MESH, "element vertex index out of range");
        if (err & kErrArea) return set_error(NLFEM_E_MESH, "element with zero area");
        if (err & kErrMaterial) return set_error(NLFEM_E_MESH, "element material outside the material table");
        const double x0 = key_to_double(red[0]), y0 = key_to_double(red[1]);
        const double x1 = key_to_double(red[2]), y1 = key_to_double(red[3]);
        const double rq = key_to_double(red[4]), rv = key_to_double(red[5]);
        const bool any = x1 >= x0 && y1 >= y0;

        // uniform grid over the barycentres -------------------------------
        // a clipped ball reaches its farthest vertex and any part of T_l
        const bool clip = clipped_ball(h->approach);
        double far = (clip ? h->poly.r_out : h->delta) + rq + (clip ? rv : 0.0);
        far = far * (1.0 + 1e-9) + 1e-300;
        h->far_reach = far;
        double reach = std::max(far, h->singular ? 2.0 * rv * (1.0 + 1e-9) : 0.0);
        h->gr = 2;
        h->gh = reach / h->gr;
        h->gx0 = any ? x0 : 0.0;
        h->gy0 = any ? y0 : 0.0;
        const double wx = any ? x1 - x0 : 0.0, wy = any ? y1 - y0 : 0.0;
        // keep the number of cells in the order of the number of elements
        for (;;) {
            const double nx = std::floor(wx / h->gh) + 1.0, ny = std::floor(wy / h->gh) + 1.0;
            if (nx * ny <= 2.0 * (double)K + 64.0) {
                h->gnx = (int32_t)nx;
                h->gny = (int32_t)ny;
                break;
            }
            h->gh *= 1.5;
        }
    }
    const int64_t ncell = (int64_t)h->gnx * h->gny;
    NLFEM_TRY(ensure_typed(h, B_CELLCNT, ncell + 1, h->cell_cnt));
    NLFEM_TRY(ensure_typed(h, B_CELLSTART, ncell + 1, h->cell_start));
    NLFEM_TRY(ensure_typed(h, B_CELLFILL, ncell, h->cell_fill));
    NLFEM_TRY(ensure_typed(h, B_CELLELEMS, K, h->cell_elems));
    NLFEM_TRY(ensure_typed(h, B_CELLOF, K, h->cell_of));
    if (!spec) {
        int bits = 0;
        while (((int64_t)1 << bits) < std::max<int64_t>(h->gnx, h->gny)) ++bits;
        h->morton_bits = ((int64_t)1 << (2 * bits)) <= 16 * ncell + 1024 ? bits : -1;
    }
    const int64_t ncode = morton_codes(h);   // <= 4 * max(gnx, gny)^2
    NLFEM_TRY(ensure_typed(h, B_NCODE, M, h->node_code));
    NLFEM_TRY(ensure_typed(h, B_CODECNT, ncode + 1, h->code_cnt));
    NLFEM_TRY(ensure_typed(h, B_CODESTART, ncode + 1, h->code_start));
    NLFEM_TRY(ensure_typed(h, B_CODEFILL, ncode, h->code_fill));
    {
        // the four scans of a build (cleared with the counters)
        const int64_t tiles[4] = {scan_tiles(M) + scan_tiles(ncell) + scan_tiles(ncode), scan_tiles(K),
                                  scan_tiles(K, kLsLast), scan_tiles(std::max(M, K))};
        int64_t words = 0;
        for (int c = 0; c < 4; ++c) words += 1 + tiles[c];
        NLFEM_TRY(ensure_typed(h, B_SCAN, words, h->scan_tmp));
        h->scan_hdr = words;
        int64_t o = 0;
        for (int c = 0; c < 4; ++c) {
            h->scan_w[c] = ScanWork{h->scan_tmp + o, tiles[c]};
            o += 1 + tiles[c];
        }
    }
    NLFEM_TRY(ensure_typed(h, B_LCNT, kLsLast * K1, h->lcnt));
    NLFEM_TRY(ensure_typed(h, B_CAND, std::max<int64_t>(K, 1), h->cand));
    NLFEM_TRY(ensure_typed(h, B_SCROFF, K1, h->scr_off));
    NLFEM_TRY(ensure_typed(h, B_LOFF, kLsLast * K1, h->loff));
    NLFEM_TRY(ensure_typed(h, B_NLEN, M + 1, h->nlen));
    NLFEM_TRY(ensure_typed(h, B_NPTR, M + 1, h->nptr));
    NLFEM_TRY(ensure_typed(h, B_NEPTR, M + 1, h->ne_ptr));
    NLFEM_TRY(ensure_typed(h, B_NELIST, 3 * K, h->ne_list));
    NLFEM_TRY(ensure_typed(h, B_NEFILL, M, h->ne_fill));
    NLFEM_TRY(ensure_typed(h, B_DOFL, M, h->dof_list));
    if (clipped_ball(h->approach)) {
        // h->poly lives as long as the handle, so the copy may run asynchronously
        NLFEM_TRY(ensure_typed(h, B_POLYDIR, 2 * kMaxPoly, h->poly_dir));
        if (h->poly.N > 0)
            NLFEM_HIP(hipMemcpyAsync(h->poly_dir, h->poly.dir, sizeof(double) * 2 * h->poly.N, hipMemcpyHostToDevice,
                                     s));
    }
    if (!spec) {
        // every counter of the rest of the build starts at zero
        ZeroList z = build_counters(h);
        z.add(h->red + kRedCounts, kRedErr - kRedCounts);   // slots 6..17, keeps the error bits
        NLFEM_TRY(launch_zero(z, nullptr, s));
    }
    // node -> element incidence, grid cells, dof rows ---------------------
    NLFEM_TRY(launch_bucket_count(h, m, s));
    {
        const ScanPart parts[3] = {{h->nlen, h->ne_ptr, M, nullptr, nullptr},
                                   {h->cell_cnt, h->cell_start, ncell, nullptr, nullptr},
                                   {h->code_cnt, h->code_start, ncode, (int64_t *)(h->red + kRedDofs), nullptr}};
        NLFEM_TRY(exclusive_scan_multi(parts, 3, h->scan_w[0], s, h->gate));
    }
    NLFEM_TRY(launch_bucket_fill(h, m, s));

    // pair search: one pass into per-element scratch segments sized by the
    // candidates, then the scan of the six per-element counts ---------------
    NLFEM_TRY(exclusive_scan(h->cand, h->scr_off, K, h->scan_w[1], s, (int64_t *)(h->red + kRedCand),
                             nullptr, h->gate));
    if (spec) {
        h->gate.mask = kSpecCand;
    } else {
        NLFEM_TRY(read_slots(h, s));
        h->total_cand = (int64_t)red[kRedCand];
    }
    NLFEM_TRY(ensure_typed(h, B_SNBRT, std::max<int64_t>(h->total_cand, 1), h->snbr_tmp));
    NLFEM_TRY(ensure_typed(h, B_SFLAGT, std::max<int64_t>(h->total_cand, 1), h->sflag_tmp));
    NLFEM_TRY(ensure_typed(h, B_SMASKT, std::max<int64_t>(h->total_cand, 1), h->smask_tmp));
    timing_begin(kPhPairs, s);
    NLFEM_TRY(launch_pairs(h, m, s));
    timing_end(kPhPairs, s);
    NLFEM_TRY(exclusive_scan_segments(h->lcnt, h->loff, K, kLsLast, K1, h->scan_w[2],
                                      (int64_t *)(h->red + kRedTot), s, (int64_t *)(h->red + kRedSegMax), h->gate));
    if (spec) {
        // list sizes, dof count and clip bound of the last build
        h->gate.mask = kSpecPairs;
    } else {
        NLFEM_TRY(read_slots(h, s));
        int64_t tot[kLsLast];
        for (int k = 0; k < kLsLast; ++k) tot[k] = (int64_t)red[kRedTot + k];
        h->max_clip = (int32_t)red[kRedClip];
        h->nS = tot[kLsS];
        h->nP = tot[kLsP];
        h->nUF = tot[kLsUF];
        h->nUTc[0] = tot[kLsUI];
        h->nUTc[1] = tot[kLsUE];
        h->nUTc[2] = tot[kLsUV];
        h->nUT = h->nUTc[0] + h->nUTc[1] + h->nUTc[2];
        h->max_S = (int64_t)red[kRedSegMax + kLsS];
        h->n_dof = (int64_t)red[kRedDofs];
        h->n_pairs = h->nP;
        h->n_ident = h->nUTc[0];
        h->n_edge = 2 * h->nUTc[1];
        h->n_vertex = 2 * h->nUTc[2];
        h->n_far = h->n_pairs - h->n_ident - h->n_edge - h->n_vertex;
        if (h->nS >= (int64_t)INT32_MAX || h->nUF >= (int64_t)INT32_MAX || h->nUT >= (int64_t)INT32_MAX)
            return set_error(NLFEM_E_OVERFLOW, "more than 2^31 neighbour entries");
        if (g_capacity > 0 && h->nS > g_capacity)
            return set_error(NLFEM_E_OVERFLOW, std::to_string(h->nS) + " neighbour entries exceed the capacity limit of " +
                                                   std::to_string(g_capacity));
    }
    NLFEM_TRY(ensure_typed(h, B_SNBR, h->nS, h->snbr));
    NLFEM_TRY(ensure_typed(h, B_SFLAG, h->nS, h->sflag));
    NLFEM_TRY(ensure_typed(h, B_SREC, h->nS, h->srec));
    NLFEM_TRY(ensure_typed(h, B_SNODE, h->nS, h->snode));
    NLFEM_TRY(ensure_typed(h, B_UE, h->nUF, h->ue));
    NLFEM_TRY(ensure_typed(h, B_UF, h->nUF, h->uf));
    NLFEM_TRY(ensure_typed(h, B_UM, h->nUF, h->um));
    NLFEM_TRY(ensure_typed(h, B_TE, h->nUT, h->te));
    NLFEM_TRY(ensure_typed(h, B_TF, h->nUT, h->tf));
    timing_begin(kPhLists, s);
    NLFEM_TRY(launch_sort_lists(h, s));
    timing_end(kPhLists, s);

    if (h->dg) return build_dg_rest(h, m, s);

    // CSR pattern -------------------------------------------------------------
    int hcap = 64;
    while (hcap < 4 * (h->max_S + 8) && hcap < 16384) hcap <<= 1;
    if (spec) hcap = h->hcap;
    for (bool links = true;; links = false) {
        h->hcap = hcap;
        NLFEM_TRY(ensure_typed(h, B_CSRSTAGE, std::max<int64_t>(h->n_dof, 1) * csr_slot(hcap), h->csr_stage));
        timing_begin(kPhCsr, s);
        NLFEM_TRY(launch_csr_rows(h, m, s, links));   // the mirror links ride on the first launch
        timing_end(kPhCsr, s);
        NLFEM_TRY(exclusive_scan(h->nlen, h->nptr, M, h->scan_w[3], s, (int64_t *)(h->red + kRedNnz),
                                 (int64_t *)(h->red + kRedMaxRow), h->gate));
        if (spec) {
            // the row capacity and nnz of the last build; the decision waits
            // for the one read-back at the end
            h->gate.mask = kSpecCsr;
            break;
        }
        NLFEM_TRY(read_slots(h, s));
        err = (int32_t)(red[kRedErr] & 0xffffffffull);
        if (!(err & kErrRowCap)) break;
        if (hcap >= 16384) return set_error(NLFEM_E_OVERFLOW, "matrix row longer than the symbolic capacity");
        hcap <<= 1;
        ZeroList z{};
        z.add(h->err, 1);
        z.add(h->red + kRedMaxRow, 1);
        z.add(h->scan_w[3].hdr, 1 + h->scan_w[3].tiles);
        NLFEM_TRY(launch_zero(z, nullptr, s));
    }
    if (err & kErrEdge) return set_error(NLFEM_E_MESH, "an edge is shared by more than two elements");
    if (err) return set_error(NLFEM_E_OVERFLOW, "internal capacity exceeded during the pair search");
    if (!spec) {
        h->nnz_node = (int64_t)red[kRedNnz];
        h->n_dof = (int64_t)red[kRedDofs];
        h->max_row = (int64_t)red[kRedMaxRow];
    }
    NLFEM_TRY(ensure_typed(h, B_NCOL, h->nnz_node, h->ncol));
    timing_begin(kPhCsr, s);
    // a rebuild's read-back: the pack launch copies the slots to the pinned
    // buffer itself
    NLFEM_TRY(launch_csr_pack(h, s, spec ? h->rb : nullptr));
    timing_end(kPhCsr, s);

    // workspace of the assembly: one result record per unordered pair
    h->far_stride = far_record_stride(h->ncomp);
    h->touch_stride = touch_record_stride(h->ncomp, h->nonsym != 0);
    double *far_rec = nullptr;
    NLFEM_TRY(ensure_typed(h, B_FARREC, h->nUF * h->far_stride, far_rec));
    h->far_rec = far_rec;
    NLFEM_TRY(ensure_typed(h, B_TOUCHREC, h->nUT * h->touch_stride, h->touch_rec));
    NLFEM_TRY(ensure_typed(h, B_DSUM, K * 6 * (h->ncomp == 1 ? 1 : 3), h->dsum));
    if (spec) {
        // the read-back (written by the pack launch) is checked by the next
        // call that uses the handle (resolve); until then assembly launches
        // test the slots themselves
        NLFEM_HIP(hipEventRecord(h->ev_rb, s));
        h->gate = SpecGate{};
        h->pending = true;
        h->pend_mesh = *m;
        h->pend_cfg.set(*cfg);
        h->pend_stream = s;
        h->asm_gate = SpecGate{h->red, h->spec_want, kSpecCsr & ~(1u << kRedErr)};
        return NLFEM_OK;
    }
    // the slots of this build, expected by the next speculative rebuild (the
    // device copy is taken from the device slots, in stream order)
    NLFEM_TRY(ensure_typed(h, B_SPEC, kRedSlots, h->spec_want));
    NLFEM_HIP(hipMemcpyAsync(h->spec_want, h->red, sizeof(unsigned long long) * kRedSlots, hipMemcpyDeviceToDevice,
                             s));
    std::memcpy(h->spec_red, red, sizeof h->spec_red);
    h->spec_ok = true;
    ++h->generation;
    return NLFEM_OK;
}

}  // namespace

int dev_alloc(DevBlock &b, size_t bytes, hipStream_t s)
{
    b = DevBlock{};
    if (!g_alloc.alloc) {
        const hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return set_error(NLFEM_E_NOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                                                " bytes failed: " + hipGetErrorString(e));
        }
    } else {
        b.p = g_alloc.alloc(bytes, (void *)s, g_alloc.ctx);
        if (!b.p)
            return set_error(NLFEM_E_NOMEM, "the allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
        b.free_fn = g_alloc.free_fn;
        b.ctx = g_alloc.ctx;
        b.stream = s;
        if ((uintptr_t)b.p & 255u) {
            dev_release(b);
            return set_error(NLFEM_E_INVALID, "the allocator hook returned memory not aligned to 256 bytes");
        }
    }
    b.cap = bytes;
    return NLFEM_OK;
}

void dev_release(DevBlock &b)
{
    if (b.p) {
        if (b.free_fn) b.free_fn(b.p, (void *)b.stream, b.ctx);
        else (void)hipFree(b.p);
    }
    b = DevBlock{};
}

// Finishes an unchecked rebuild: waits for its read-back and, when the sizes
// differ, counts the assemblies queued since (their kernels skipped their
// work) and runs the plain build of the rebuild's mesh.
int resolve(nlfem_pairs *h)
{
    if (!h->pending) return NLFEM_OK;
    h->pending = false;
    h->asm_gate = SpecGate{};
    NLFEM_TRY(wait_event(h->ev_rb));
    const int64_t queued = h->pend_asm;
    h->pend_asm = 0;
    if (rebuild_held(h)) return NLFEM_OK;
    h->skipped += queued;
    h->last_build = 2;
    int rc = build(&h->pend_mesh, &h->pend_cfg.c, h, h->pend_stream, false);
    if (rc == NLFEM_OK) {
        // the plain build's last launches are still queued on its stream
        NLFEM_HIP(hipEventRecord(h->ev_rb, h->pend_stream));
        rc = wait_event(h->ev_rb);
    }
    if (rc != NLFEM_OK) {
        h->spec_ok = false;
        h->gate = SpecGate{};
        h->K = 0;   // unusable rather than half built
    }
    return rc;
}

namespace {

// same sizes and the same configuration of the pair search as the handle
bool same_shape(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *c)
{
    if (h->M != m->n_vertices || h->K != m->n_elements) return false;
    if (h->kernel != c->kernel || h->approach != c->approach || h->delta != c->delta) return false;
    if (h->singular != (c->singular_n > 0)) return false;
    if (h->dg != (c->ansatz == NLFEM_ANSATZ_DG)) return false;
    if (h->materials != c->n_materials) return false;
    if (h->nonsym != (c->n_materials > 0 && material_nonsymmetric(c))) return false;
    const RuleArgs r = make_rules(c);
    if (r.P != h->rules.P || r.Q != h->rules.Q) return false;
    if (std::memcmp(r.pxi, h->rules.pxi, sizeof r.pxi) || std::memcmp(r.pw, h->rules.pw, sizeof r.pw) ||
        std::memcmp(r.qxi, h->rules.qxi, sizeof r.qxi) || std::memcmp(r.qw, h->rules.qw, sizeof r.qw))
        return false;
    if (clipped_ball(c->approach)) {
        const PolyArgs p = make_poly(c);
        if (p.N != h->poly.N || std::memcmp(p.dir, h->poly.dir, sizeof p.dir)) return false;
    }
    return true;
}

bool same_build(const nlfem_pairs *h, const nlfem_mesh *m, const nlfem_config *c)
{
    if (h->mesh_vertices != m->vertices || h->mesh_elements != m->elements || h->mesh_labels != m->labels)
        return false;
    if (c->n_materials > 0 && h->mesh_materials != m->materials) return false;
    return same_shape(h, m, c);
}

}  // namespace

// ---- timing
namespace {
struct Timing {
    bool on = false;
    int mask = 0;                 // bit p: phase p is timed
    static constexpr int kPool = 4096;
    hipEvent_t ev[kPool];
    int used = 0;
    int open_slot[kPhLast];
    struct Pair {
        int phase, a, b;
    };
    Pair pairs[kPool / 2];
    int npairs = 0;
    double ms[kPhLast] = {};
    int64_t launches[kPhLast] = {};
};
Timing g_timing;

int timing_collect()
{
    for (int k = 0; k < g_timing.npairs; ++k) {
        const auto &p = g_timing.pairs[k];
        float ms = 0.f;
        NLFEM_HIP(hipEventSynchronize(g_timing.ev[p.b]));
        NLFEM_HIP(hipEventElapsedTime(&ms, g_timing.ev[p.a], g_timing.ev[p.b]));
        g_timing.ms[p.phase] += ms;
        g_timing.launches[p.phase] += 1;
    }
    g_timing.npairs = 0;
    g_timing.used = 0;
    return NLFEM_OK;
}
}  // namespace

void timing_begin(int phase, hipStream_t s)
{
    if (!g_timing.on || !((g_timing.mask >> phase) & 1)) return;
    if (g_timing.used + 2 > Timing::kPool) timing_collect();
    const int a = g_timing.used++;
    g_timing.open_slot[phase] = a;
    (void)hipEventRecord(g_timing.ev[a], s);
}

void timing_end(int phase, hipStream_t s)
{
    if (!g_timing.on || !((g_timing.mask >> phase) & 1)) return;
    const int b = g_timing.used++;
    (void)hipEventRecord(g_timing.ev[b], s);
    g_timing.pairs[g_timing.npairs++] = {phase, g_timing.open_slot[phase], b};
}

int set_error(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NLFEM_E_NOMEM : NLFEM_E_HIP;
}

}  // namespace nlfem

using namespace nlfem;

extern "C" {

int32_t nlfem_version(void) { return NLFEM_ABI_VERSION; }

const char *nlfem_last_error(void) { return g_err.c_str(); }

int nlfem_build_pairs(const nlfem_mesh *mesh, const nlfem_config *cfg, nlfem_pairs **pairs, void *stream)
{
    if (!pairs) return set_error(NLFEM_E_INVALID, "pairs is NULL");
    NLFEM_TRY(check_mesh(mesh));
    NLFEM_TRY(check_cfg(cfg));
    if (cfg->n_materials > 0 && !mesh->materials)
        return set_error(NLFEM_E_INVALID, "mesh materials are NULL with a material table");
    NLFEM_TRY(check_device());
    const bool fresh = *pairs == nullptr;
    nlfem_pairs *h = fresh ? new (std::nothrow) nlfem_pairs() : *pairs;
    if (!h) return set_error(NLFEM_E_NOMEM, "host allocation failed");
    bool held = true;
    if (!fresh && h->pending) {
        // a newer build replaces an unchecked one: its read-back is checked
        // (assemblies queued after it skipped their work if it failed), but
        // its plain build is not run
        NLFEM_TRY(wait_event(h->ev_rb));
        h->pending = false;
        h->asm_gate = SpecGate{};
        held = rebuild_held(h);
        if (!held) h->skipped += h->pend_asm;
        h->pend_asm = 0;
    }
    // after a rebuild that found other sizes the mesh has probably changed:
    // build plainly
    const bool spec = !fresh && held && h->spec_ok && same_shape(h, mesh, cfg) && cfg->ansatz == NLFEM_ANSATZ_CG;
    int rc = build(mesh, cfg, h, (hipStream_t)stream, spec);
    h->last_build = spec ? 1 : 0;
    if (rc != NLFEM_OK) {
        h->spec_ok = false;
        h->gate = SpecGate{};
        if (fresh) nlfem_pairs_free(h);
        else h->K = 0;   // leave a reused handle unusable rather than half built
        return rc;
    }
    *pairs = h;
    return NLFEM_OK;
}

int nlfem_pairs_info(const nlfem_pairs *h, nlfem_pairs_info_t *info)
{
    if (!h || !info) return set_error(NLFEM_E_INVALID, "NULL argument");
    NLFEM_TRY(resolve(const_cast<nlfem_pairs *>(h)));
    info->n_pairs = h->n_pairs;
    info->n_far = h->n_far;
    info->n_vertex = h->n_vertex;
    info->n_edge = h->n_edge;
    info->n_ident = h->n_ident;
    info->n_dof = h->n_dof;
    info->n_rows = h->n_dof * h->ncomp;
    info->nnz = h->nnz_node * h->ncomp * h->ncomp;
    info->n_upper_far = h->nUF;
    info->n_upper_touch = h->nUT;
    info->n_nbr = h->nS;
    info->rebuild = h->last_build;
    info->skipped = h->skipped;
    return NLFEM_OK;
}

int nlfem_pairs_export(const nlfem_pairs *h, int32_t *k, int32_t *l, int8_t *cls, void *stream)
{
    if (h) NLFEM_TRY(resolve(const_cast<nlfem_pairs *>(h)));
    if (!h || h->K == 0) return set_error(NLFEM_E_INVALID, "pairs handle is NULL or not built");
    if (h->n_pairs > 0 && (!k || !l || !cls)) return set_error(NLFEM_E_INVALID, "NULL output array");
    return launch_export(h, k, l, cls, (hipStream_t)stream);
}

int nlfem_csr_pattern(const nlfem_pairs *h, int64_t *row_ptr, int32_t *col, void *stream)
{
    if (h) NLFEM_TRY(resolve(const_cast<nlfem_pairs *>(h)));
    if (!h || h->K == 0) return set_error(NLFEM_E_INVALID, "pairs handle is NULL or not built");
    if (!row_ptr || (h->nnz_node > 0 && !col)) return set_error(NLFEM_E_INVALID, "NULL output array");
    if (h->dg) return launch_dg_pattern(h, row_ptr, col, (hipStream_t)stream);
    return launch_pattern(h, row_ptr, col, (hipStream_t)stream);
}

int nlfem_assemble(const nlfem_mesh *mesh, const nlfem_config *cfg, const nlfem_pairs *h, double *val,
                   void *stream)
{
    if (!h || h->K == 0) return set_error(NLFEM_E_INVALID, "pairs handle is NULL or not built");
    NLFEM_TRY(check_mesh(mesh));
    NLFEM_TRY(check_cfg(cfg));
    if (cfg->n_materials > 0 && !mesh->materials)
        return set_error(NLFEM_E_INVALID, "mesh materials are NULL with a material table");
    if (h->nnz_node > 0 && !val) return set_error(NLFEM_E_INVALID, "val is NULL");
    if (!same_build(h, mesh, cfg))
        return set_error(NLFEM_E_MISMATCH, "mesh or configuration differs from the one the pairs were built for");
    int dev = -1;
    NLFEM_HIP(hipGetDevice(&dev));
    if (dev != h->device) return set_error(NLFEM_E_MISMATCH, "current device differs from the build device");
    GaussArgs g{};
    g.n = cfg->singular_n;
    if (g.n > 0) gauss_legendre01(g.n, g.x, g.w);
    // after an unchecked rebuild the launches test its slots on the device
    // (asm_gate) and skip their work when they differ; the check of the
    // read-back is left to the next call that needs the sizes
    if (h->pending) ++const_cast<nlfem_pairs *>(h)->pend_asm;
    return launch_assemble(h, mesh, cfg, g, val, (hipStream_t)stream);
}

int nlfem_rhs(const nlfem_mesh *mesh, const nlfem_config *cfg, const double *f_qp, const double *f_affine,
              double *b, void *stream)
{
    NLFEM_TRY(check_mesh(mesh));
    if (!cfg) return set_error(NLFEM_E_INVALID, "config is NULL");
    if (cfg->kernel < NLFEM_K_CONSTANT || cfg->kernel > NLFEM_K_FRAC_HALF)
        return set_error(NLFEM_E_INVALID, "unknown kernel");
    NLFEM_TRY(check_rule(cfg->outer, "outer"));
    if (!b) return set_error(NLFEM_E_INVALID, "b is NULL");
    if (!f_qp && !f_affine) return set_error(NLFEM_E_INVALID, "give f_qp or f_affine");
    const int nc = ncomp_of(cfg->kernel);
    if (!f_qp)
        for (int t = 0; t < 3 * nc; ++t)
            if (!is_finite(f_affine[t])) return set_error(NLFEM_E_INVALID, "f_affine not finite");
    NLFEM_TRY(check_device());
    timing_begin(kPhRhs, (hipStream_t)stream);
    if (cfg->ansatz != NLFEM_ANSATZ_CG && cfg->ansatz != NLFEM_ANSATZ_DG)
        return set_error(NLFEM_E_INVALID, "unknown ansatz");
    const int rc = launch_rhs(mesh, make_rules(cfg), nc, f_qp, f_affine, b, (hipStream_t)stream,
                              cfg->ansatz == NLFEM_ANSATZ_DG);
    timing_end(kPhRhs, (hipStream_t)stream);
    return rc;
}

int nlfem_timing_enable(int mask)
{
    if (mask < 0 || mask >= (1 << NLFEM_TIMING_PHASES))
        return set_error(NLFEM_E_INVALID, "timing mask has bits outside the phases");
    const bool on = mask != 0;
    if (on && g_timing.on) NLFEM_TRY(timing_collect());   // close the pairs of the old mask
    g_timing.mask = mask;
    if (on && !g_timing.on) {
        NLFEM_TRY(check_device());
        for (int k = 0; k < Timing::kPool; ++k) NLFEM_HIP(hipEventCreate(&g_timing.ev[k]));
        g_timing.used = g_timing.npairs = 0;
        for (int k = 0; k < kPhLast; ++k) {
            g_timing.ms[k] = 0.0;
            g_timing.launches[k] = 0;
        }
        g_timing.on = true;
    } else if (!on && g_timing.on) {
        NLFEM_TRY(timing_collect());
        for (int k = 0; k < Timing::kPool; ++k) (void)hipEventDestroy(g_timing.ev[k]);
        g_timing.on = false;
    }
    return NLFEM_OK;
}

int nlfem_timing_read(double *ms, int64_t *launches, int reset)
{
    if (!ms || !launches) return set_error(NLFEM_E_INVALID, "NULL output array");
    if (g_timing.on) NLFEM_TRY(timing_collect());
    for (int k = 0; k < kPhLast; ++k) {
        ms[k] = g_timing.ms[k];
        launches[k] = g_timing.launches[k];
        if (reset) {
            g_timing.ms[k] = 0.0;
            g_timing.launches[k] = 0;
        }
    }
    return NLFEM_OK;
}

int nlfem_set_allocator(nlfem_alloc_fn alloc, nlfem_free_fn free_, void *ctx)
{
    if ((alloc == nullptr) != (free_ == nullptr))
        return set_error(NLFEM_E_INVALID, "give both allocator functions or neither");
    g_alloc = Allocator{alloc, free_, alloc ? ctx : nullptr};
    return NLFEM_OK;
}

int nlfem_set_capacity(int64_t max_entries)
{
    if (max_entries < 0) return set_error(NLFEM_E_INVALID, "capacity must be >= 0");
    g_capacity = max_entries;
    return NLFEM_OK;
}

void nlfem_pairs_free(nlfem_pairs *h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();   // no queued work may still use the buffers
    for (auto &b : h->bufs) dev_release(b);
    if (h->rb) (void)hipHostFree(h->rb);
    if (h->ev_rb) (void)hipEventDestroy(h->ev_rb);
    delete h;
}

}  // extern "C"

namespace {

// checks a batch's problems and makes their launch plans; handles with an
// unchecked rebuild are finished first when `resolve_pending`, rejected
// otherwise (finishing one may run a plain build, which allocates)
int batch_plans(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs, nlfem_pairs *const *pairs,
                double *const *vals, bool resolve_pending, std::vector<items::AssemblePlan> &plans,
                std::vector<nlfem_pairs *> &handles)
{
    if (n < 1 || n > NLFEM_MAX_BATCH) return set_error(NLFEM_E_INVALID, "batch size outside [1, NLFEM_MAX_BATCH]");
    if (!meshes || !cfgs || !pairs || !vals) return set_error(NLFEM_E_INVALID, "NULL array argument");
    NLFEM_TRY(check_device());
    int dev = -1;
    NLFEM_HIP(hipGetDevice(&dev));
    plans.reserve(n);
    for (int i = 0; i < n; ++i) {
        nlfem_pairs *h = pairs[i];
        if (h && h->pending) {
            if (!resolve_pending)
                return set_error(NLFEM_E_INVALID, "pairs handle " + std::to_string(i) +
                                                      " has an unchecked rebuild (call nlfem_pairs_info first)");
            NLFEM_TRY(resolve(h));
        }
        if (!h || h->K == 0) return set_error(NLFEM_E_INVALID, "pairs handle " + std::to_string(i) + " is NULL or not built");
        NLFEM_TRY(check_mesh(&meshes[i]));
        NLFEM_TRY(check_cfg(&cfgs[i]));
        if (cfgs[i].n_materials > 0 && !meshes[i].materials)
            return set_error(NLFEM_E_INVALID, "mesh materials are NULL with a material table");
        if (material_nonsymmetric(&cfgs[i]))
            return set_error(NLFEM_E_INVALID,
                             "batches take symmetric material tables (a non-symmetric one runs in the "
                             "single-problem path)");
        if (h->nnz_node > 0 && !vals[i]) return set_error(NLFEM_E_INVALID, "val " + std::to_string(i) + " is NULL");
        if (!same_build(h, &meshes[i], &cfgs[i]))
            return set_error(NLFEM_E_MISMATCH, "problem " + std::to_string(i) +
                                                   ": mesh or configuration differs from the one its pairs were built for");
        if (dev != h->device) return set_error(NLFEM_E_MISMATCH, "current device differs from a build device");
        if (h->dg) return set_error(NLFEM_E_INVALID, "batches take problems of the continuous ansatz");
        if (kernel_variant(&cfgs[i]) & kKerNoZeroDiv)
            return set_error(NLFEM_E_INVALID,
                             "batches take singular kernels with singular_n > 0 (the no-zero-division rule runs "
                             "in the single-problem path)");
        for (int j = 0; j < i; ++j)
            if (pairs[j] == h) return set_error(NLFEM_E_INVALID, "a pairs handle appears twice (shared workspace)");
        GaussArgs g{};
        g.n = cfgs[i].singular_n;
        if (g.n > 0) gauss_legendre01(g.n, g.x, g.w);
        plans.push_back(items::make_plan(h, &meshes[i], &cfgs[i], g, vals[i]));
        handles.push_back(h);
    }
    return NLFEM_OK;
}

}  // namespace

extern "C" {

int nlfem_batch_create(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs, nlfem_pairs *const *pairs,
                       double *const *vals, const char *tune_cache, int32_t tune, nlfem_batch **batch,
                       void *stream)
{
    if (!batch) return set_error(NLFEM_E_INVALID, "batch is NULL");
    *batch = nullptr;
    if (tune < 0 || tune > 2) return set_error(NLFEM_E_INVALID, "tune must be 0, 1 or 2");
    std::vector<items::AssemblePlan> plans;
    std::vector<nlfem_pairs *> handles;
    NLFEM_TRY(batch_plans(n, meshes, cfgs, pairs, vals, true, plans, handles));
    return batch_create(plans, handles, tune_cache, tune, batch, (hipStream_t)stream);
}

int nlfem_assemble_batched_noalloc(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs,
                                   nlfem_pairs *const *pairs, double *const *vals, void *stream)
{
    std::vector<items::AssemblePlan> plans;
    std::vector<nlfem_pairs *> handles;
    NLFEM_TRY(batch_plans(n, meshes, cfgs, pairs, vals, false, plans, handles));
    return batch_assemble_noalloc(plans, (hipStream_t)stream);
}

int nlfem_batch_assemble(nlfem_batch *batch, void *stream)
{
    if (!batch) return set_error(NLFEM_E_INVALID, "batch is NULL");
    return batch_run(batch, (hipStream_t)stream);
}

int nlfem_batch_launch_graph(nlfem_batch *batch, void *stream)
{
    if (!batch) return set_error(NLFEM_E_INVALID, "batch is NULL");
    return batch_graph_launch(batch, (hipStream_t)stream);
}

int nlfem_batch_info(const nlfem_batch *batch, int32_t *groups, int32_t *shape)
{
    if (!batch || !groups || !shape) return set_error(NLFEM_E_INVALID, "NULL argument");
    return batch_info(batch, groups, shape);
}

void nlfem_batch_free(nlfem_batch *batch) { batch_free(batch); }

int nlfem_assemble_batched(int32_t n, const nlfem_mesh *meshes, const nlfem_config *cfgs, nlfem_pairs *const *pairs,
                           double *const *vals, const char *tune_cache, void *stream)
{
    nlfem_batch *b = nullptr;
    NLFEM_TRY(nlfem_batch_create(n, meshes, cfgs, pairs, vals, tune_cache, tune_cache ? 1 : 0, &b, stream));
    int rc = batch_run(b, (hipStream_t)stream);
    if (rc == NLFEM_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        rc = set_error(NLFEM_E_HIP, "hipStreamSynchronize");
    batch_free(b);
    return rc;
}

}  // extern "C"
