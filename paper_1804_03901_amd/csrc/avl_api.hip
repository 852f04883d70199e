// libavl host side: configuration checks, workspace layout, launch order of
// the time step (Sec. 2, Fig. "algorithm"), HIP-graph replay and timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/avl.h"
#include "avl_device.h"

namespace avl {
hipError_t launch_sort(const Geo& g, void* src, void* dst, const double* E, const RowShift* rows, double dtk,
                       float bk, int* counts, int* offsets, int* tile_sums, int* tile_next, int* flags, bool push,
                       hipStream_t st, int phase, const int* off_old, const int* tf_old, int* tf_new);
hipError_t launch_cells(const Geo& g, const int* offsets, int* cell, hipStream_t st);
hipError_t launch_push(const Geo& g, void* m, const double* E, const RowShift* rows, double dtk, float bk,
                       int* flags, hipStream_t st);
hipError_t launch_recon(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid, double* rho_part,
                        hipStream_t st);
int recon_capacity(int prec);
hipError_t launch_recon3(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid, double* rho_part,
                         void* scratch, hipStream_t st);
hipError_t launch_field(const Geo& g, const double* rho_part, const double* rho_in, double* rho_slices, double* rho,
                        double* E_out, const double2* tw, const double* green, double* diag_ring,
                        long long* step_ctr, int write_diag, double* W_out, int* flags, hipStream_t st);
int field_slices(const Geo& g);
hipError_t launch_rho_slices(const Geo& g, const double* rho_part, double* rho_slices, hipStream_t st);
hipError_t launch_species_rho(const Species* sp, int ns, int nx, int from_rho, double* rho_total, hipStream_t st);
hipError_t launch_broadcast_E(const Species* sp, int ns, int nx, hipStream_t st);
hipError_t launch_validate(const Geo& g, const double* x, const double* v, const double* f, int* bad,
                           hipStream_t st);
hipError_t launch_to32(const Geo& g, const double* x, const double* v, const double* f, M32 m, int* flags,
                       hipStream_t st);
hipError_t launch_to64(const Geo& g, M32 m, double* x, double* v, double* f, hipStream_t st,
                       const int* id = nullptr);
hipError_t launch_by_id64(int n, const double* x, const double* v, const int* id, double* xo, double* vo,
                          hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
size_t recon3_scratch_bytes(const Geo& g);
hipError_t launch_iota(int* id, int n, hipStream_t st);
hipError_t launch_adj_deposit(const Geo& g, int grid_prec, const double* x, const double* v, const int* id,
                              const double* f_by_id, const void* fg, const void* Dg, const double* R, double rscale,
                              double* lam_x, double* lam_v, double* f_bar, int with_positions, hipStream_t st);
hipError_t launch_adj_step_rev(const Geo& g, int grid_prec, const double* x1, const double* v1, const double* f_by_id,
                               const void* fg, const void* Dg, const double* R, double rscale, const double* x0,
                               const double* E0, double c, double* lam_x, double* lam_v, double* f_bar,
                               unsigned long long* acc, unsigned* key, hipStream_t st);
hipError_t launch_adj_push(const Geo& g, const double* x, const int* id, const double* E, double c,
                           const double* lam_x_in, const double* lam_v_in, double* lam_x, double* lam_v,
                           unsigned long long* acc, unsigned* key, hipStream_t st);
hipError_t launch_adj_mu(const Geo& g, const double* E, double w, unsigned long long* acc, unsigned* key, double* mu,
                         hipStream_t st);
hipError_t launch_adj_clear(int nx, unsigned long long* acc, unsigned* key, hipStream_t st);
hipError_t launch_fill_f64(double* p, int n, double value, hipStream_t st);
hipError_t launch_scale_f64(double* p, int n, double s, hipStream_t st);
int sort_blocks(const Geo& g, int phase);
size_t sort_lds(const Geo& g);
size_t scatter_lds(const Geo& g);
int recon_waves_per_cu(int prec, int lds_per_cu);
int scatter_blocks_per_cu(const Geo& g);
int scatter_step_blocks_per_cu(const Geo& g);
int count_blocks_per_cu(const Geo& g);
int diag_chunks(const Geo& g);
hipError_t launch_diag(const Geo& g, const void* fgrid, const double* rho, const double* E, double mass,
                       double* part, double* out, double* j_out, double* drho_out, hipStream_t st);
hipError_t launch_sort_batch(int prec, const BInst* tab, const int* pre, int ninst, int blocks, size_t smem, int cur,
                             hipStream_t st, int phase);
bool recon_sparse(const Geo& g);
hipError_t launch_recon_batch(int prec, int kahan, int sparse, const BInst* tab, const int* pre, int ninst, int tasks, int cur,
                              hipStream_t st);
hipError_t launch_field_batch(const BInst* tab, const int* pre, int ninst, int rho_blocks, int max_nx, int write_diag,
                              hipStream_t st);
void set_lds_limit(int bytes);
}  // namespace avl

using namespace avl;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t markers[2], counts, offsets[2], tfirst[2], tile_sums, fgrid, rho_part, rho_slices, rho, E, tw, green, rows, diag, ctr, flags, bad,
        scratch3, diag_part, adj, total;
};

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Compute units of the current device (256 on MI355X, assumed when no device
// is visible, so that sizes computed without a GPU match).
int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return cus;
}

// LDS bytes of one compute unit (160 KB on MI355X, assumed when no device is
// visible).
int device_lds_per_cu()
{
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds <= 0) {
        (void)hipGetLastError();
        return 160 * 1024;
    }
    return lds;
}

// Grids of the tiled FP32 1D-1V sort passes: the blocks that fit on every
// compute unit at once, at most sort_cap per compute unit when that is set.
// A pass that is not tiled reports 0 (a block per tile) and stays 0.
void sort_launch_shapes(Geo& g)
{
    const int cus = device_cus();
    auto capped = [&](int per_cu) { return g.sort_cap > 0 ? std::min(per_cu, g.sort_cap) : per_cu; };
    g.sblocks = capped(scatter_blocks_per_cu(g)) * cus;
    g.sblocks_step = capped(scatter_step_blocks_per_cu(g)) * cus;
    g.cblocks = capped(count_blocks_per_cu(g)) * cus;
}

// Validate a configuration and derive the kernel constants.
int make_geo(const avl_config* c, Geo* g)
{
    if (!c) return AVL_EINVAL;
    std::memset(g, 0, sizeof(Geo));
    if (c->vdim != 1 && c->vdim != 3) return AVL_EINVAL;
    if (c->nx < 8 || c->nx > kMaxNx || (c->nx & (c->nx - 1))) return AVL_EINVAL;
    if (c->precision != AVL_FP64 && c->precision != AVL_FP32) return AVL_EINVAL;
    if (c->first_kick != 0 && c->first_kick != 1) return AVL_EINVAL;
    if (c->options & ~AVL_OPT_KAHAN32) return AVL_EINVAL;
    if (c->tune[0] < 0 || c->tune[0] > 256 || c->tune[1] < 0 || c->tune[1] > 2 || c->tune[2] < 0 ||
        c->tune[2] > 64 || c->tune[3])
        return AVL_EINVAL;
    if ((c->options & AVL_OPT_KAHAN32) && c->precision != AVL_FP32) return AVL_EINVAL;
    // the 1D-3V reconstruction always accumulates in FP64
    if ((c->options & AVL_OPT_KAHAN32) && c->vdim == 3) return AVL_ENOTSUP;
    if (c->n_markers < 0 || c->n_markers >= (int64_t)INT32_MAX) return AVL_ESIZE;
    if (!finite_pos(c->L) || !finite_pos(c->dt) || !finite_pos(c->c_p)) return AVL_EINVAL;
    if (!std::isfinite(c->q) || !std::isfinite(c->m) || c->m == 0.0) return AVL_EINVAL;
    {
        // background magnetic field: 1D-3V only; at least 2 pi steps per gyration
        const bool any = c->B[0] != 0.0 || c->B[1] != 0.0 || c->B[2] != 0.0;
        if (!std::isfinite(c->B[0]) || !std::isfinite(c->B[1]) || !std::isfinite(c->B[2])) return AVL_EINVAL;
        if (any && c->vdim != 3) return AVL_EINVAL;
        const double wc = std::fabs(c->q / c->m) * std::sqrt(c->B[0] * c->B[0] + c->B[1] * c->B[1] + c->B[2] * c->B[2]);
        if (wc * c->dt > 1.0) return AVL_EINVAL;
        if (any && c->precision == AVL_FP32) return AVL_ENOTSUP;
        g->magnetic = any ? 1 : 0;
        for (int d = 0; d < 3; ++d) g->B[d] = c->B[d];
    }
    g->vdim = c->vdim;
    g->prec = c->precision;
    g->kahan = (c->options & AVL_OPT_KAHAN32) ? 1 : 0;
    g->sort_cap = c->tune[2];
    g->nx = c->nx;
    g->lognx = ilog2(c->nx);
    int64_t rows = 1, cells = c->nx;
    double vol = 1.0;
    for (int d = 0; d < c->vdim; ++d) {
        if (c->nv[d] < 2 || c->nv[d] > (1 << 20)) return AVL_EINVAL;
        if (!std::isfinite(c->vmin[d]) || !std::isfinite(c->vmax[d]) || !(c->vmax[d] > c->vmin[d]))
            return AVL_EINVAL;
        g->nv[d] = c->nv[d];
        rows *= (c->nv[d] + 1);
        cells *= c->nv[d];
        // each factor is at most 2^20 + 1: checking after every one keeps
        // the products far inside int64
        if (rows * c->nx >= (int64_t)INT32_MAX || cells >= (int64_t)INT32_MAX) return AVL_ESIZE;
        g->vmin[d] = c->vmin[d];
        g->dv[d] = (c->vmax[d] - c->vmin[d]) / c->nv[d];
        g->inv_dv[d] = 1.0 / g->dv[d];
        vol *= g->dv[d];
    }
    for (int d = c->vdim; d < 3; ++d) g->nv[d] = 1;
    if (rows * c->nx + 2 >= (int64_t)INT32_MAX || cells >= (int64_t)INT32_MAX) return AVL_ESIZE;
    // the 1D-1V reconstruction addresses each marker array with 32-bit byte offsets
    if (c->vdim == 1 && (c->n_markers + 64) * (c->precision == AVL_FP64 ? 8 : 4) > (int64_t)0xffffffffLL)
        return AVL_ESIZE;
    g->nrow = (int)rows;
    g->nb = (int)(rows * c->nx);
    g->n = (int)c->n_markers;
    g->np = (int)((c->n_markers + 63) / 64 * 64);
    g->L = c->L;
    g->inv_L = 1.0 / c->L;
    g->dx = c->L / c->nx;
    g->inv_dx = 1.0 / g->dx;
    g->dt = c->dt;
    g->qm = c->q / c->m;
    g->cp = c->c_p;
    g->q_vol = c->q * vol;
    g->bscale = (float)(g->qm * c->dt * g->inv_dv[0]);
    g->gam = (float)(g->dv[0] * c->dt * g->inv_dx);
    g->c0f = (float)(c->vmin[0] * g->inv_dv[0] + 0.5);
    // sort window: the bucket rows one count tile spans, plus one each side
    {
        const double per_row = rows > 0 ? (double)c->n_markers / (double)rows : 0.0;
        const double span = per_row > 0 ? (double)kCountTile / per_row : 1.0;
        int64_t want = (int64_t)(std::ceil(span) + 3) * c->nx;
        want = std::max<int64_t>(want, 4 * (int64_t)c->nx);
        want = std::min<int64_t>(want, std::max<int64_t>(8192, 4 * (int64_t)c->nx));
        g->hist_bins = (int)want;
        // the step's scatter (2048-marker tiles, a row or two of buckets in
        // the dense rows) keeps three rows: a tile inside one row and its
        // neighbours, which leaves room for five blocks per CU
        g->sbins = (int)std::min<int64_t>(g->hist_bins, std::max<int64_t>(3 * (int64_t)c->nx, kSortTile));
    }
    // reconstruction decomposition
    if (c->vdim == 1) {
        // wave tasks of one 63-column strip by rc velocity rows: the fewest
        // rows per task such that all tasks are resident at once (as many
        // waves as the reconstruction's registers and LDS let a compute unit
        // hold), so there is no partial second round; tune[0] overrides rc
        g->nstrip = (c->nx + kReconCols - 1) / kReconCols;
        const int64_t slots =
            (int64_t)recon_waves_per_cu(c->precision == AVL_FP32 ? 1 : 0, device_lds_per_cu()) * device_cus();
        int rc = 2;
        while (rc < 32 && (int64_t)g->nstrip * ((c->nv[0] + rc - 1) / rc) > slots) ++rc;
        if (c->tune[0]) rc = c->tune[0];
        g->rc = rc;
        g->rform = c->tune[1];
        g->nchunk = (c->nv[0] + rc - 1) / rc;
        g->cap = recon_capacity(c->precision);
    } else {
        // 1D-3V FP32 encoding of the x-velocity dual index: jrange is a power
        // of two (the kernels decode it with a mask and a shift)
        int jr = 1;
        while (jr < c->nv[0] + 1 + 64) jr <<= 1;
        g->jrange = jr;
        g->jpad = (jr - (c->nv[0] + 1)) / 2;
        if (c->precision == AVL_FP32 &&
            (int64_t)jr * (c->nv[1] + 1) * (c->nv[2] + 1) * c->nx >= (int64_t)INT32_MAX)
            return AVL_ESIZE;
        // one wave task per 63-column strip and target (vy, vz) plane; the rho
        // partials are per plane
        g->nstrip = (c->nx + kReconCols - 1) / kReconCols;
        g->rc = 1;
        g->nchunk = c->nv[1] * c->nv[2];
        g->cap = 0;
    }
    return AVL_OK;
}

void make_layout(const avl_config* c, const Geo& g, Layout* L)
{
    size_t n = (size_t)g.np;
    size_t mbytes = c->precision == AVL_FP64 ? sizeof(double) * n * (2 + g.vdim) : 4 * n * (3 + g.vdim);
    size_t esz = c->precision == AVL_FP64 ? 8 : 4;
    size_t cells = (size_t)g.nx;
    for (int d = 0; d < g.vdim; ++d) cells *= g.nv[d];
    size_t nbt = (size_t)g.nb + 1;
    size_t ntiles = (nbt + kScanTile - 1) / kScanTile;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L->markers[0] = take(mbytes + 64 * (3 + g.vdim));
    L->markers[1] = take(mbytes + 64 * (3 + g.vdim));
    L->counts = take(sizeof(int) * nbt);
    // run offsets and tile-start buckets of each marker buffer's order
    L->offsets[0] = take(sizeof(int) * (nbt + 1));
    L->offsets[1] = take(sizeof(int) * (nbt + 1));
    L->tfirst[0] = take(sizeof(int) * (n / 2048 + 2));
    L->tfirst[1] = take(sizeof(int) * (n / 2048 + 2));
    L->tile_sums = take(sizeof(int) * 2 * (ntiles + 64));   // two parities of per-tile totals
    L->fgrid = take(esz * cells);
    L->rho_part = take(sizeof(double) * (size_t)std::max(1, g.nchunk) * g.nx);
    L->rho_slices = take(sizeof(double) * (size_t)kMaxFieldSlices * g.nx);
    L->rho = take(sizeof(double) * g.nx);
    L->E = take(sizeof(double) * g.nx);
    L->tw = take(sizeof(double) * g.nx);
    L->green = take(sizeof(double) * g.nx);
    L->rows = take(sizeof(RowShift) * (g.nv[0] + 1));
    L->diag = take(sizeof(double) * 2 * kDiagCap);
    L->ctr = take(sizeof(long long));
    L->flags = take(sizeof(int));
    L->bad = take(sizeof(int));
    L->scratch3 = take(g.vdim == 3 ? recon3_scratch_bytes(g) : 0);
    L->diag_part = take(sizeof(double) * 4 * (size_t)g.nx * diag_chunks(g));
    // reverse runs: integer sums of the field adjoint (2 nx), their bound key
    L->adj = take(sizeof(unsigned long long) * 2 * (size_t)g.nx + 256);
    L->total = off;
}

// Shrink LDS-sized parameters to what one block may use on this device.
void fit_lds(Geo* g, int lds)
{
    const int esz = 8;                    // staged field: double, or the FP32 form's (kick, difference) pair
    if (g->vdim == 1) g->cap = recon_capacity(g->prec);
    const int fixed = esz * g->nx + (g->prec ? (int)sizeof(RowShift) * (g->nv[0] + 1) : 0) + 64;
    int bins = (lds - fixed) / 4;
    bins = (bins >> g->lognx) << g->lognx;
    if (g->hist_bins > bins) g->hist_bins = bins;
    if (g->sbins > g->hist_bins) g->sbins = g->hist_bins;
}

}  // namespace

struct avl_handle {
    avl_config cfg;
    Geo g;
    Layout lay;
    hipStream_t st;
    char* ws;
    M64 m64[2];
    M32 m32[2];
    int cur;
    int *counts, *offsets, *tile_sums, *flags, *bad;
    int *offs[2], *tfirst[2];   // run offsets / tile-start buckets of each marker buffer's order; offsets = offs[cur]
    bool cells_ok;      // FP32 1D-1V: every stored cell index is current (else implied by offs[cur])
    void* fgrid;
    double *rho_part, *rho_slices, *rho, *E, *green, *diag;
    double2* tw;
    RowShift* rows;
    long long* ctr;
    void* scratch3;
    bool sorted, have_f, have_rho, have_E;
    bool partials;      // rho partials of the current markers are in the workspace
    bool kicked;        // a push has happened since loading (first-kick rule)
    int64_t steps;      // steps enqueued since loading (mirrors the device counter)
    hipGraphExec_t gexec[2];
    hipStream_t cap_st;   // capture stream (the legacy default stream cannot be captured)
    bool graph_ok;
    bool timing;
    void* rec_D;        // adjoint runs: the step's reconstruction also writes D here
    std::vector<hipEvent_t> ev[AVL_K_COUNT];
    size_t ev_used[AVL_K_COUNT];
};

namespace {

void* marker_view(avl_handle* h, int which)
{
    return h->g.prec == AVL_FP64 ? (void*)&h->m64[which] : (void*)&h->m32[which];
}

void set_views(avl_handle* h)
{
    const size_t n = (size_t)h->g.np;
    for (int b = 0; b < 2; ++b) {
        char* p = h->ws + h->lay.markers[b];
        if (h->g.prec == AVL_FP64) {
            double* d = reinterpret_cast<double*>(p);
            h->m64[b].x = d;
            h->m64[b].v = d + n;
            h->m64[b].f = d + n * (1 + h->g.vdim);
            h->m64[b].id = nullptr;
        } else {
            int* c = reinterpret_cast<int*>(p);
            h->m32[b].cell = c;
            h->m32[b].a = reinterpret_cast<float*>(c + n);
            h->m32[b].b = reinterpret_cast<float*>(c + 2 * n);
            h->m32[b].f = reinterpret_cast<float*>(c + n * (2 + h->g.vdim));
            h->m32[b].id = nullptr;
        }
    }
}

int hip_status(hipError_t e) { return e == hipSuccess ? AVL_OK : AVL_EDEVICE; }

bool debug_on()
{
    static int on = -1;
    if (on < 0) on = std::getenv("AVL_DEBUG") ? 1 : 0;
    return on == 1;
}

int report(hipError_t e, const char* what, int line)
{
    if (debug_on()) std::fprintf(stderr, "[avl] %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
    return AVL_EDEVICE;
}

#define AVL_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return report(e_, #expr, __LINE__); \
    } while (0)

}  // namespace

namespace avl {
KernelEvents& pending_events()
{
    static thread_local KernelEvents e{nullptr, nullptr};
    return e;
}
}  // namespace avl

namespace {

// Events around one phase of a step on the library's stream.  A phase that is
// one kernel launched through launch() (attach) hands its pair to that launch,
// which then records the kernel's own start and end; if no launch took the
// pair (nothing to do), both are recorded at once.
struct Timer {
    avl_handle* h;
    int k;
    hipEvent_t start, stop;
    bool attach;
    Timer(avl_handle* hh, int kk, bool single_kernel = false)
        : h(hh), k(kk), start(nullptr), stop(nullptr), attach(single_kernel)
    {
        if (!h->timing) return;
        std::vector<hipEvent_t>& v = h->ev[k];
        if (h->ev_used[k] + 2 > v.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                v.push_back(e);
            }
        }
        start = v[h->ev_used[k]];
        stop = v[h->ev_used[k] + 1];
        h->ev_used[k] += 2;
        if (attach) pending_events() = KernelEvents{start, stop};
        else (void)hipEventRecord(start, h->st);
    }
    ~Timer()
    {
        if (!stop) return;
        if (attach) {
            KernelEvents& pe = pending_events();
            if (pe.start != start) return;          // taken by the phase's kernel
            pe = KernelEvents{nullptr, nullptr};
            (void)hipEventRecord(start, h->st);
        }
        (void)hipEventRecord(stop, h->st);
    }
};

double kick_fraction(avl_handle* h) { return (!h->kicked && h->cfg.first_kick) ? 0.5 : 1.0; }

// Host tables: FFT twiddles, the field solve's transfer function and the FP32
// drift table; written into the workspace at load time.
int upload_tables(avl_handle* h)
{
    const Geo& g = h->g;
    const int nx = g.nx;
    std::vector<double> tw(nx), green(nx);
    for (int k = 0; k < nx / 2; ++k) {
        const double ang = 2.0 * M_PI * (double)k / (double)nx;
        tw[2 * k] = std::cos(ang);
        tw[2 * k + 1] = -std::sin(ang);
    }
    // Eq. (kappasoftening): kappa = k sinc(k dx), K^2 = k^2 sinc^2(k dx / 2)
    for (int m = 0; m < nx; ++m) {
        if (m == 0 || 2 * m == nx) { green[m] = 0.0; continue; }
        const int mp = (2 * m < nx) ? m : m - nx;
        const double k = 2.0 * M_PI * mp / g.L;
        const double y = k * g.dx;
        const double kappa = k * (std::sin(y) / y);
        const double s = std::sin(0.5 * y) / (0.5 * y);
        const double K2 = k * k * s * s;
        green[m] = g.cp * kappa / K2;
    }
    std::vector<RowShift> rows(g.nv[0] + 1);
    for (int jp = 0; jp <= g.nv[0]; ++jp) {
        const double vel = g.vmin[0] + ((double)(jp - 1) + 0.5) * g.dv[0];
        const double P = vel * g.dt / g.dx;
        double w = std::floor(P);
        float fr = (float)(P - w);
        if (fr >= 1.0f) { fr = 0.0f; w += 1.0; }
        rows[jp].whole = (int)w;
        rows[jp].frac = fr;
    }
    AVL_TRY(hipMemcpyAsync(h->tw, tw.data(), sizeof(double) * nx, hipMemcpyHostToDevice, h->st));
    AVL_TRY(hipMemcpyAsync(h->green, green.data(), sizeof(double) * nx, hipMemcpyHostToDevice, h->st));
    AVL_TRY(hipMemcpyAsync(h->rows, rows.data(), sizeof(RowShift) * rows.size(), hipMemcpyHostToDevice, h->st));
    AVL_TRY(hipStreamSynchronize(h->st));
    return AVL_OK;
}

bool implied_cells(const avl_handle* h) { return h->g.prec == AVL_FP32 && h->g.vdim == 1; }

// FP32 1D-1V: write the cell index of every marker of a sorted order (the
// sort stores it only for the overflow bucket), before anything that reads
// the cells outside a sort (export, an order-preserving push, a raw copy).
int ensure_cells(avl_handle* h)
{
    if (!implied_cells(h) || h->cells_ok) return AVL_OK;
    AVL_TRY(launch_cells(h->g, h->offsets, h->m32[h->cur].cell, h->st));
    h->cells_ok = true;
    return AVL_OK;
}

int do_sort(avl_handle* h, bool push, double kick)
{
    const Geo& g = h->g;
    void* src = marker_view(h, h->cur);
    void* dst = marker_view(h, 1 - h->cur);
    const double dtk = g.dt * kick;
    const float bk = g.bscale * (float)kick;
    // per-scan-tile totals alternate between two halves with the buffer parity
    const size_t tstride = ((size_t)g.nb + 1 + kScanTile - 1) / kScanTile + 64;
    int* tcur = h->tile_sums + (size_t)h->cur * tstride;
    int* tnext = h->tile_sums + (size_t)(1 - h->cur) * tstride;
    // FP32 1D-1V markers in a sorted order carry implied cells
    const bool impl = implied_cells(h) && h->sorted;
    const int* off_old = impl ? h->offs[h->cur] : nullptr;
    const int* tf_old = impl ? h->tfirst[h->cur] : nullptr;
    int* off_new = h->offs[1 - h->cur];
    int* tf_new = h->tfirst[1 - h->cur];
    {
        Timer t(h, AVL_K_PUSH_COUNT, true);
        AVL_TRY(launch_sort(g, src, dst, h->E, h->rows, dtk, bk, h->counts, off_new, tcur, tnext, h->flags,
                            push, h->st, 0, off_old, tf_old, tf_new));
    }
    {
        Timer t(h, AVL_K_SCAN);
        AVL_TRY(launch_sort(g, src, dst, h->E, h->rows, dtk, bk, h->counts, off_new, tcur, tnext, h->flags,
                            push, h->st, 1, off_old, tf_old, tf_new));
    }
    {
        Timer t(h, AVL_K_SCATTER, true);
        AVL_TRY(launch_sort(g, src, dst, h->E, h->rows, dtk, bk, h->counts, off_new, tcur, tnext, h->flags,
                            push, h->st, 2, off_old, tf_old, tf_new));
    }
    h->cur = 1 - h->cur;
    h->offsets = h->offs[h->cur];
    h->cells_ok = !implied_cells(h);
    h->sorted = true;
    if (push) {
        h->kicked = true;
        h->have_f = h->have_rho = h->have_E = h->partials = false;
    }
    return AVL_OK;
}

// Reconstruction of f (the kernel also writes per-chunk column partials of
// the rho moment, which the field kernel adds in chunk order).
int do_recon(avl_handle* h, void* Dgrid)
{
    {
        Timer t(h, AVL_K_RECONSTRUCT, true);
        if (h->g.vdim == 1)
            AVL_TRY(launch_recon(h->g, marker_view(h, h->cur), h->offsets, h->fgrid, Dgrid, h->rho_part, h->st));
        else
            AVL_TRY(launch_recon3(h->g, marker_view(h, h->cur), h->offsets, h->fgrid, Dgrid, h->rho_part,
                                  h->scratch3, h->st));
    }
    // rho stays valid when the markers have not moved since it was formed
    if (!h->have_f) h->have_rho = false;
    h->have_f = true;
    h->partials = true;
    return AVL_OK;
}

// rho from the partials (or the caller's rho) and the field solve, one launch.
int do_field(avl_handle* h, const double* rho_in, bool diag, double* W_out)
{
    Timer t(h, AVL_K_FIELD);
    if (!rho_in && !h->partials) return AVL_ESTATE;
    AVL_TRY(launch_field(h->g, h->rho_part, rho_in, h->rho_slices, h->rho, h->E, h->tw, h->green, h->diag, h->ctr,
                         diag ? 1 : 0, W_out, h->flags, h->st));
    if (!rho_in) h->have_rho = true;
    h->have_E = true;
    return AVL_OK;
}

int one_step(avl_handle* h)
{
    Timer t(h, AVL_K_STEP);
    int rc = do_sort(h, true, kick_fraction(h));
    if (rc) return rc;
    if ((rc = do_recon(h, h->rec_D))) return rc;
    if ((rc = do_field(h, nullptr, true, nullptr))) return rc;
    h->steps += 1;
    return AVL_OK;
}

// Load FP64 markers into buffer `cur` (converting to the FP32 form if needed),
// validate them, and rebuild f, rho, E.
int load_markers(avl_handle* h, const double* x, const double* v, const double* f, bool fresh)
{
    const Geo& g = h->g;
    const size_t n = (size_t)g.n;
    if (n > 0 && (!x || !v || !f)) return AVL_EINVAL;
    if (((uintptr_t)x | (uintptr_t)v | (uintptr_t)f) & 7) return AVL_EALIGN;
    AVL_TRY(hipMemsetAsync(h->bad, 0, sizeof(int), h->st));
    AVL_TRY(launch_validate(g, x, v, f, h->bad, h->st));
    int bad = 0;
    AVL_TRY(hipMemcpyAsync(&bad, h->bad, sizeof(int), hipMemcpyDeviceToHost, h->st));
    AVL_TRY(hipStreamSynchronize(h->st));
    if (bad) return AVL_EINVAL;
    h->cur = 0;
    if (n == 0) {
        // nothing to copy
    } else if (g.prec == AVL_FP64) {
        AVL_TRY(hipMemcpyAsync(h->m64[0].x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, h->st));
        for (int d = 0; d < g.vdim; ++d)
            AVL_TRY(hipMemcpyAsync(h->m64[0].v + (size_t)d * g.np, v + (size_t)d * n, sizeof(double) * n,
                                   hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(h->m64[0].f, f, sizeof(double) * n, hipMemcpyDeviceToDevice, h->st));
        // adjoint runs: identities are the positions in the caller's order
        if (h->m64[0].id) AVL_TRY(launch_iota(h->m64[0].id, (int)n, h->st));
    } else {
        AVL_TRY(launch_to32(g, x, v, f, h->m32[0], h->flags, h->st));
        if (h->m32[0].id) AVL_TRY(launch_iota(h->m32[0].id, (int)n, h->st));
    }
    const int total = g.n;
    const size_t nbt = (size_t)g.nb + 1;
    AVL_TRY(hipMemsetAsync(h->counts, 0, sizeof(int) * nbt, h->st));
    {
        const size_t ntiles = (nbt + kScanTile - 1) / kScanTile;
        AVL_TRY(hipMemsetAsync(h->tile_sums, 0, sizeof(int) * 2 * (ntiles + 64), h->st));
    }
    AVL_TRY(hipMemcpyAsync(h->offs[0] + nbt, &total, sizeof(int), hipMemcpyHostToDevice, h->st));
    AVL_TRY(hipMemcpyAsync(h->offs[1] + nbt, &total, sizeof(int), hipMemcpyHostToDevice, h->st));
    if (fresh) AVL_TRY(hipMemsetAsync(h->ctr, 0, sizeof(long long), h->st));
    AVL_TRY(hipStreamSynchronize(h->st));
    if (fresh) {
        h->steps = 0;
        h->kicked = false;
    }
    h->sorted = false;
    h->cells_ok = true;
    h->offsets = h->offs[0];
    h->have_f = h->have_rho = h->have_E = h->partials = false;
    int rc;
    if ((rc = do_sort(h, false, 1.0))) return rc;
    if ((rc = do_recon(h, nullptr))) return rc;
    if ((rc = do_field(h, nullptr, false, nullptr))) return rc;
    return AVL_OK;
}

void drop_graphs(avl_handle* h)
{
    for (int b = 0; b < 2; ++b)
        if (h->gexec[b]) {
            (void)hipGraphExecDestroy(h->gexec[b]);
            h->gexec[b] = nullptr;
        }
    h->graph_ok = false;
}

int copy_diag(avl_handle* h, int64_t first, int32_t count, double* out)
{
    int64_t done = 0;
    while (done < count) {
        int64_t pos = (first + done) % kDiagCap;
        int64_t len = std::min<int64_t>(count - done, kDiagCap - pos);
        AVL_TRY(hipMemcpyAsync(out + 2 * done, h->diag + 2 * pos, sizeof(double) * 2 * len, hipMemcpyDeviceToDevice,
                               h->st));
        done += len;
    }
    return AVL_OK;
}

}  // namespace

extern "C" {

size_t avl_workspace_bytes(const avl_config* cfg)
{
    Geo g;
    if (make_geo(cfg, &g) != AVL_OK) return 0;
    Layout L;
    make_layout(cfg, g, &L);
    return L.total;
}

int avl_init(const avl_config* cfg, void* workspace, size_t ws_bytes, void* stream, const double* x,
             const double* v, const double* f, avl_handle** out)
{
    if (!out) return AVL_EINVAL;
    *out = nullptr;
    Geo g;
    int rc = make_geo(cfg, &g);
    if (rc) return rc;
    Layout lay;
    make_layout(cfg, g, &lay);
    if (!workspace) return AVL_EINVAL;
    if ((uintptr_t)workspace % kAlign) return AVL_EALIGN;
    if (ws_bytes < lay.total) return AVL_ESIZE;
    avl_handle* h = new (std::nothrow) avl_handle();
    if (!h) return AVL_EINVAL;
    h->cfg = *cfg;
    h->g = g;
    h->lay = lay;
    h->st = (hipStream_t)stream;
    h->ws = (char*)workspace;
    set_views(h);
    h->counts = (int*)(h->ws + lay.counts);
    for (int b = 0; b < 2; ++b) {
        h->offs[b] = (int*)(h->ws + lay.offsets[b]);
        h->tfirst[b] = (int*)(h->ws + lay.tfirst[b]);
    }
    h->offsets = h->offs[0];
    h->cells_ok = true;
    h->tile_sums = (int*)(h->ws + lay.tile_sums);
    h->fgrid = h->ws + lay.fgrid;
    h->rho_part = (double*)(h->ws + lay.rho_part);
    h->rho_slices = (double*)(h->ws + lay.rho_slices);
    h->rho = (double*)(h->ws + lay.rho);
    h->E = (double*)(h->ws + lay.E);
    h->tw = (double2*)(h->ws + lay.tw);
    h->green = (double*)(h->ws + lay.green);
    h->rows = (RowShift*)(h->ws + lay.rows);
    h->diag = (double*)(h->ws + lay.diag);
    h->ctr = (long long*)(h->ws + lay.ctr);
    h->flags = (int*)(h->ws + lay.flags);
    h->bad = (int*)(h->ws + lay.bad);
    h->scratch3 = h->ws + lay.scratch3;
    h->gexec[0] = h->gexec[1] = nullptr;
    h->cap_st = nullptr;
    {
        // size LDS use from what the device lets one block opt into
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) != hipSuccess) { delete h; return AVL_EDEVICE; }
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || lds <= 0)
            if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
        set_lds_limit(lds);
        fit_lds(&h->g, lds);
        sort_launch_shapes(h->g);
        if (debug_on())
            std::fprintf(stderr,
                         "[avl] lds limit %d B, recon cap %d, hist bins %d, rc %d, chunks %d, strips %d, "
                         "recon waves per CU %d\n",
                         lds, h->g.cap, h->g.hist_bins, h->g.rc, h->g.nchunk, h->g.nstrip,
                         h->g.vdim == 1 ? recon_waves_per_cu(h->g.prec, device_lds_per_cu()) : 0);
    }
    if (hipMemsetAsync(h->flags, 0, sizeof(int), h->st) != hipSuccess || (rc = upload_tables(h)) != AVL_OK) {
        delete h;
        return rc ? rc : AVL_EDEVICE;
    }
    rc = load_markers(h, x, v, f, true);
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return AVL_OK;
}

int avl_push(avl_handle* h, const double* E)
{
    if (!h) return AVL_EINVAL;
    if (!E && !h->have_E) return AVL_ESTATE;
    const double kick = kick_fraction(h);
    int rc0 = ensure_cells(h);
    if (rc0) return rc0;
    {
        Timer t(h, AVL_K_PUSH_COUNT);
        AVL_TRY(launch_push(h->g, marker_view(h, h->cur), E ? E : h->E, h->rows, h->g.dt * kick,
                            h->g.bscale * (float)kick, h->flags, h->st));
    }
    h->kicked = true;
    h->sorted = false;
    h->have_f = h->have_rho = h->have_E = h->partials = false;
    return AVL_OK;
}

int avl_sort(avl_handle* h)
{
    if (!h) return AVL_EINVAL;
    return do_sort(h, false, 1.0);
}

int avl_reconstruct(avl_handle* h, void* f_out, void* D_out)
{
    if (!h) return AVL_EINVAL;
    int rc;
    if (!h->sorted && (rc = do_sort(h, false, 1.0))) return rc;
    if ((rc = do_recon(h, D_out))) return rc;
    if (f_out) {
        size_t cells = (size_t)h->g.nx;
        for (int d = 0; d < h->g.vdim; ++d) cells *= h->g.nv[d];
        AVL_TRY(hipMemcpyAsync(f_out, h->fgrid, cells * (h->g.prec ? 4 : 8), hipMemcpyDeviceToDevice, h->st));
    }
    return AVL_OK;
}

int avl_moments(avl_handle* h, double* rho_out)
{
    if (!h) return AVL_EINVAL;
    if (!h->have_f) return AVL_ESTATE;
    if (!h->have_rho) {
        // forming rho also solves the field from it (one fused launch)
        int rc = do_field(h, nullptr, false, nullptr);
        if (rc) return rc;
    }
    if (rho_out) AVL_TRY(hipMemcpyAsync(rho_out, h->rho, sizeof(double) * h->g.nx, hipMemcpyDeviceToDevice, h->st));
    return AVL_OK;
}

int avl_poisson(avl_handle* h, const double* rho, double* E_out, double* W_out)
{
    if (!h) return AVL_EINVAL;
    if (!rho && !h->have_f && !h->have_rho) return AVL_ESTATE;
    int rc = do_field(h, rho ? rho : (h->have_rho ? h->rho : nullptr), false, W_out);
    if (rc) return rc;
    if (E_out) AVL_TRY(hipMemcpyAsync(E_out, h->E, sizeof(double) * h->g.nx, hipMemcpyDeviceToDevice, h->st));
    return AVL_OK;
}

int avl_step(avl_handle* h, int32_t nsteps, double* diag_out)
{
    if (!h) return AVL_EINVAL;
    if (nsteps < 0) return AVL_EINVAL;
    if (!h->have_E || !h->sorted) return AVL_ESTATE;
    int64_t first = h->steps;
    for (int32_t s = 0; s < nsteps; ++s) {
        int rc = one_step(h);
        if (rc) return rc;
        if (diag_out && ((s + 1) % kDiagCap == 0)) {
            if ((rc = copy_diag(h, first + s + 1 - kDiagCap, kDiagCap, diag_out + 2 * (s + 1 - kDiagCap)))) return rc;
        }
    }
    if (diag_out) {
        int32_t tail = nsteps % kDiagCap;
        if (tail) return copy_diag(h, first + nsteps - tail, tail, diag_out + 2 * (nsteps - tail));
    }
    return AVL_OK;
}

int avl_step_graph(avl_handle* h, int32_t nsteps, double* diag_out)
{
    if (!h) return AVL_EINVAL;
    if (nsteps < 0) return AVL_EINVAL;
    if (!h->have_E || !h->sorted) return AVL_ESTATE;
    if (h->timing) return avl_step(h, nsteps, diag_out);
    int64_t first = h->steps;
    int32_t s = 0;
    // a half first kick is a different launch argument: run it directly
    if (nsteps > 0 && kick_fraction(h) != 1.0) {
        int rc = one_step(h);
        if (rc) return rc;
        s = 1;
    }
    if (!h->graph_ok && s < nsteps) {
        // capture one step from each buffer parity on a side stream; the graph
        // is then launched on the handle's stream
        if (!h->cap_st) AVL_TRY(hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking));
        AVL_TRY(hipStreamSynchronize(h->st));
        const hipStream_t user_st = h->st;
        for (int b = 0; b < 2; ++b) {
            hipGraph_t graph = nullptr;
            const int saved_cur = h->cur;
            const int64_t saved_steps = h->steps;
            h->cur = b;
            h->st = h->cap_st;
            hipError_t e = hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal);
            int rc = e == hipSuccess ? one_step(h) : AVL_EDEVICE;
            hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(h->st, &graph) : e;
            h->st = user_st;
            h->cur = saved_cur;
            h->steps = saved_steps;
            h->offsets = h->offs[h->cur];
            if (e != hipSuccess) return report(e, "hipStreamBeginCapture", __LINE__);
            if (e2 != hipSuccess) return report(e2, "hipStreamEndCapture", __LINE__);
            if (rc) return rc;
            e = hipGraphInstantiate(&h->gexec[b], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                drop_graphs(h);
                return report(e, "hipGraphInstantiate", __LINE__);
            }
        }
        h->graph_ok = true;
    }
    for (; s < nsteps; ++s) {
        AVL_TRY(hipGraphLaunch(h->gexec[h->cur], h->st));
        h->cur = 1 - h->cur;
        h->offsets = h->offs[h->cur];
        h->cells_ok = !implied_cells(h);
        h->steps += 1;
        if (diag_out && ((s + 1) % kDiagCap == 0)) {
            int rc = copy_diag(h, first + s + 1 - kDiagCap, kDiagCap, diag_out + 2 * (s + 1 - kDiagCap));
            if (rc) return rc;
        }
    }
    h->sorted = true;
    h->have_f = h->have_rho = h->have_E = h->partials = true;
    h->kicked = true;
    if (diag_out) {
        int32_t tail = nsteps % kDiagCap;
        if (tail) return copy_diag(h, first + nsteps - tail, tail, diag_out + 2 * (nsteps - tail));
    }
    return AVL_OK;
}

int avl_get_markers(avl_handle* h, double* x, double* v, double* f)
{
    if (!h) return AVL_EINVAL;
    const Geo& g = h->g;
    const size_t n = (size_t)g.n;
    if (n == 0) return AVL_OK;
    if (!x || !v || !f) return AVL_EINVAL;
    if (((uintptr_t)x | (uintptr_t)v | (uintptr_t)f) & 7) return AVL_EALIGN;
    if (g.prec == AVL_FP64) {
        const M64& m = h->m64[h->cur];
        AVL_TRY(hipMemcpyAsync(x, m.x, sizeof(double) * n, hipMemcpyDeviceToDevice, h->st));
        for (int d = 0; d < g.vdim; ++d)
            AVL_TRY(hipMemcpyAsync(v + (size_t)d * n, m.v + (size_t)d * g.np, sizeof(double) * n,
                                   hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(f, m.f, sizeof(double) * n, hipMemcpyDeviceToDevice, h->st));
        return AVL_OK;
    }
    const int rc = ensure_cells(h);
    if (rc) return rc;
    return hip_status(launch_to64(g, h->m32[h->cur], x, v, f, h->st));
}

int avl_set_markers(avl_handle* h, const double* x, const double* v, const double* f)
{
    if (!h) return AVL_EINVAL;
    drop_graphs(h);
    return load_markers(h, x, v, f, false);
}

int avl_get_field(avl_handle* h, double* E_out, double* rho_out)
{
    if (!h) return AVL_EINVAL;
    if (E_out) {
        if (!h->have_E) return AVL_ESTATE;
        AVL_TRY(hipMemcpyAsync(E_out, h->E, sizeof(double) * h->g.nx, hipMemcpyDeviceToDevice, h->st));
    }
    if (rho_out) {
        if (!h->have_rho) return AVL_ESTATE;
        AVL_TRY(hipMemcpyAsync(rho_out, h->rho, sizeof(double) * h->g.nx, hipMemcpyDeviceToDevice, h->st));
    }
    return AVL_OK;
}

int avl_diagnostics(avl_handle* h, double* out, double* j_out, double* drho_out)
{
    if (!h || !out) return AVL_EINVAL;
    if (!h->have_f || !h->have_rho || !h->have_E) return AVL_ESTATE;
    AVL_TRY(launch_diag(h->g, h->fgrid, h->rho, h->E, h->cfg.m, (double*)(h->ws + h->lay.diag_part), out, j_out,
                        drho_out, h->st));
    return AVL_OK;
}

int64_t avl_step_count(const avl_handle* h) { return h ? h->steps : -1; }

int avl_check(avl_handle* h)
{
    if (!h) return AVL_EINVAL;
    int fl = 0;
    AVL_TRY(hipMemcpyAsync(&fl, h->flags, sizeof(int), hipMemcpyDeviceToHost, h->st));
    AVL_TRY(hipStreamSynchronize(h->st));
    if (fl & FLAG_NONFINITE) return AVL_ENONFINITE;
    if (fl & (FLAG_SLOT | FLAG_RANGE)) return AVL_EINTERNAL;
    return AVL_OK;
}

int avl_status(avl_handle* h) { return avl_check(h); }

int avl_set_stream(avl_handle* h, void* stream)
{
    if (!h) return AVL_EINVAL;
    h->st = (hipStream_t)stream;
    return AVL_OK;
}

int avl_timing(avl_handle* h, int enable)
{
    if (!h) return AVL_EINVAL;
    h->timing = enable != 0;
    for (int k = 0; k < AVL_K_COUNT; ++k) h->ev_used[k] = 0;
    return AVL_OK;
}

int avl_kernel_time(avl_handle* h, int kernel, double* ms_total, int64_t* launches)
{
    if (!h || kernel < 0 || kernel >= AVL_K_COUNT) return AVL_EINVAL;
    AVL_TRY(hipStreamSynchronize(h->st));
    double tot = 0.0;
    const size_t used = h->ev_used[kernel];
    for (size_t i = 0; i + 1 < used; i += 2) {
        float ms = 0.0f;
        AVL_TRY(hipEventElapsedTime(&ms, h->ev[kernel][i], h->ev[kernel][i + 1]));
        tot += ms;
    }
    if (ms_total) *ms_total = tot;
    if (launches) *launches = (int64_t)(used / 2);
    return AVL_OK;
}

double avl_kernel_bytes(const avl_handle* h, int kernel)
{
    if (!h) return 0.0;
    const Geo& g = h->g;
    const double n = g.n;
    double cells = g.nx;
    for (int d = 0; d < g.vdim; ++d) cells *= g.nv[d];
    const bool implied = g.prec == AVL_FP32 && g.vdim == 1;     // the sort stores no cell index
    // stored bytes per marker: everything, and the position/velocity part alone
    const double mk = g.prec == AVL_FP64 ? 8.0 * (2 + g.vdim) : 4.0 * (3 + g.vdim) - (implied ? 4.0 : 0.0);
    const double pos = g.prec == AVL_FP64 ? 8.0 * (1 + g.vdim) : 4.0 * (2 + g.vdim) - (implied ? 4.0 : 0.0);
    // what the push itself must read and write: the FP32 1D-3V form moves
    // cell, a and b_x only (b_y, b_z never change)
    const double moved = (g.prec == AVL_FP32 && g.vdim == 3) ? 12.0 : pos;
    const double esz = g.prec == AVL_FP64 ? 8.0 : 4.0;
    const double runs = 4.0 * (g.nb + 1.0);                     // one run offset per bucket
    // the reconstruction reads every marker's offsets and f (the FP32 form's
    // cell index is implied by the sorted order), the run offsets, and writes
    // the f grid
    const double recon = n * (g.prec == AVL_FP64 ? mk : 4.0 * (2 + g.vdim)) + runs + cells * esz;
    switch (kernel) {
    case AVL_K_PUSH_COUNT: return n * moved + (implied ? runs : 0.0);   // positions read (+ old run offsets)
    case AVL_K_SCAN: return 3.0 * runs;                         // counts read twice, offsets written
    case AVL_K_SCATTER: return 2.0 * n * mk + (implied ? runs : 0.0);   // every marker read and written
    case AVL_K_RECONSTRUCT: return recon;
    case AVL_K_FIELD: return 8.0 * g.nx * (g.nchunk + 2.0);     // chunk partials in, rho and E out
    // the method's own bytes per step, sorting excluded: the push reads and
    // writes positions and velocities, the reconstruction as above
    case AVL_K_STEP: return 2.0 * n * moved + recon;
    default: return 0.0;
    }
}

int avl_copy_probe(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src || (bytes % 16)) return AVL_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) & 15) return AVL_EALIGN;
    return hip_status(launch_copy(src, dst, bytes, (hipStream_t)stream));
}

const char* avl_strerror(int status)
{
    switch (status) {
    case AVL_OK: return "ok";
    case AVL_EINVAL: return "invalid argument or configuration";
    case AVL_ESIZE: return "size out of range or workspace too small";
    case AVL_EALIGN: return "misaligned pointer";
    case AVL_ESTATE: return "call not valid in the current state";
    case AVL_EDEVICE: return "HIP runtime error";
    case AVL_ENOTSUP: return "configuration not supported";
    case AVL_ENONFINITE: return "non-finite value seen on the device";
    case AVL_EINTERNAL: return "device consistency check failed";
    default: return "unknown status";
    }
}

int avl_destroy(avl_handle* h)
{
    if (!h) return AVL_EINVAL;
    drop_graphs(h);
    if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
    for (int k = 0; k < AVL_K_COUNT; ++k)
        for (hipEvent_t e : h->ev[k]) (void)hipEventDestroy(e);
    delete h;
    return AVL_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent 1D-1V instances
// ---------------------------------------------------------------------------

struct avl_batch {
    int n;
    std::vector<avl_handle*> h;
    hipStream_t st;
    BInst* tab;                 // device
    int* pre;                   // device, BPRE_KINDS x (n+1)
    int tot[BPRE_KINDS];
    int prec, kahan, max_nx;
    size_t lds, lds_scatter;
    hipGraphExec_t gexec[2];
    hipStream_t cap_st;
    bool graph_ok;
};

namespace {

constexpr int kMaxBatch = 4096;

// Byte offsets of the instances' workspace slices and of the batch tables.
bool batch_layout(const avl_config* cfgs, int32_t count, std::vector<size_t>* off, size_t* tab_off, size_t* pre_off,
                  size_t* total)
{
    if (!cfgs || count < 1 || count > kMaxBatch) return false;
    size_t o = 0;
    off->assign(count, 0);
    for (int i = 0; i < count; ++i) {
        if (cfgs[i].vdim != 1) return false;
        if (cfgs[i].precision != cfgs[0].precision || cfgs[i].options != cfgs[0].options ||
            cfgs[i].first_kick != cfgs[0].first_kick)
            return false;
        Geo g;
        if (make_geo(&cfgs[i], &g) != AVL_OK) return false;
        // the batched scan takes each tile's prefix from its predecessors directly
        if ((g.nb + 1 + kScanTile - 1) / kScanTile > 1024) return false;
        Layout L;
        make_layout(&cfgs[i], g, &L);
        (*off)[i] = o;
        o = align_up(o + L.total);
    }
    *tab_off = o;
    o = align_up(o + sizeof(BInst) * (size_t)count);
    *pre_off = o;
    o = align_up(o + sizeof(int) * BPRE_KINDS * ((size_t)count + 1));
    *total = o;
    return true;
}

void drop_batch_graphs(avl_batch* b)
{
    for (int k = 0; k < 2; ++k)
        if (b->gexec[k]) {
            (void)hipGraphExecDestroy(b->gexec[k]);
            b->gexec[k] = nullptr;
        }
    b->graph_ok = false;
}

// One step of every instance: six batched launches on `st`, from buffer parity cur.
int batch_launch(avl_batch* b, int cur, hipStream_t st)
{
    AVL_TRY(launch_sort_batch(b->prec, b->tab, b->pre, b->n, b->tot[BPRE_COUNT], b->lds, cur, st, 0));
    AVL_TRY(launch_sort_batch(b->prec, b->tab, b->pre, b->n, b->tot[BPRE_SCAN], b->lds, cur, st, 1));
    AVL_TRY(launch_sort_batch(b->prec, b->tab, b->pre, b->n, b->tot[BPRE_SCATTER], b->lds_scatter, cur, st, 2));
    // the sparse-row kernels when every instance with markers has sparse rows
    bool sparse = true;
    for (avl_handle* hi : b->h)
        if (hi->g.n > 0 && !recon_sparse(hi->g)) sparse = false;
    AVL_TRY(launch_recon_batch(b->prec, b->kahan, sparse ? 1 : 0, b->tab, b->pre, b->n, b->tot[BPRE_RECON], 1 - cur,
                               st));
    AVL_TRY(launch_field_batch(b->tab, b->pre, b->n, b->tot[BPRE_RHO], b->max_nx, 1, st));
    return AVL_OK;
}

// Host-side state of the instances after a batched step.
void batch_advance(avl_batch* b)
{
    for (avl_handle* h : b->h) {
        h->cur = 1 - h->cur;
        h->offsets = h->offs[h->cur];
        h->cells_ok = !implied_cells(h);
        h->steps += 1;
        h->sorted = h->kicked = true;
        h->have_f = h->have_rho = h->have_E = h->partials = true;
    }
}

}  // namespace

extern "C" {

size_t avl_batch_workspace_bytes(const avl_config* cfgs, int32_t count)
{
    std::vector<size_t> off;
    size_t tab_off, pre_off, total;
    return batch_layout(cfgs, count, &off, &tab_off, &pre_off, &total) ? total : 0;
}

int avl_batch_init(const avl_config* cfgs, int32_t count, void* workspace, size_t ws_bytes, void* stream,
                   const double* x, const double* v, const double* f, avl_batch** out)
{
    if (!out || !workspace) return AVL_EINVAL;
    *out = nullptr;
    std::vector<size_t> off;
    size_t tab_off, pre_off, total;
    if (!batch_layout(cfgs, count, &off, &tab_off, &pre_off, &total)) {
        // tell unsupported shapes from invalid ones
        for (int i = 0; cfgs && i < count && i < kMaxBatch; ++i) {
            Geo g;
            const int rc = make_geo(&cfgs[i], &g);
            if (rc) return rc;
        }
        return (count < 1 || count > kMaxBatch || !cfgs) ? AVL_EINVAL : AVL_ENOTSUP;
    }
    if ((uintptr_t)workspace & 255) return AVL_EALIGN;
    if (ws_bytes < total) return AVL_ESIZE;
    avl_batch* b = new avl_batch();
    b->n = count;
    b->st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    int64_t mo = 0;
    for (int i = 0; i < count; ++i) {
        avl_handle* h = nullptr;
        Geo g;
        make_geo(&cfgs[i], &g);
        Layout L;
        make_layout(&cfgs[i], g, &L);
        const int64_t n = cfgs[i].n_markers;
        const int rc = avl_init(&cfgs[i], ws + off[i], L.total, stream, x ? x + mo : nullptr, v ? v + mo : nullptr,
                                f ? f + mo : nullptr, &h);
        if (rc) {
            for (avl_handle* q : b->h) avl_destroy(q);
            delete b;
            return rc;
        }
        b->h.push_back(h);
        mo += n;
    }
    // instance table and work-item prefixes
    std::vector<BInst> tab(count);
    std::vector<int> pre(BPRE_KINDS * (size_t)(count + 1), 0);
    b->prec = cfgs[0].precision;
    b->kahan = (cfgs[0].options & AVL_OPT_KAHAN32) ? 1 : 0;
    b->max_nx = 0;
    b->lds = 0;
    b->lds_scatter = 0;
    for (int i = 0; i < count; ++i) {
        avl_handle* h = b->h[i];
        const Geo& g = h->g;
        BInst& I = tab[i];
        std::memset(&I, 0, sizeof(BInst));
        I.g = g;
        for (int p = 0; p < 2; ++p) {
            I.m64[p] = h->m64[p];
            I.m32[p] = h->m32[p];
        }
        I.E = h->E;
        I.rows = h->rows;
        I.counts = h->counts;
        for (int p = 0; p < 2; ++p) {
            I.offsets[p] = h->offs[p];
            I.tfirst[p] = h->tfirst[p];
        }
        const size_t tstride = ((size_t)g.nb + 1 + kScanTile - 1) / kScanTile + 64;
        I.tsum[0] = h->tile_sums;
        I.tsum[1] = h->tile_sums + tstride;
        I.fgrid = h->fgrid;
        I.rho_part = h->rho_part;
        I.rho_slices = h->rho_slices;
        I.rho = h->rho;
        I.tw = h->tw;
        I.green = h->green;
        I.diag = h->diag;
        I.ctr = h->ctr;
        I.flags = h->flags;
        I.dtk = g.dt;
        I.bk = g.bscale;
        I.nslice = field_slices(g);
        const int items[BPRE_KINDS] = {sort_blocks(g, 0), sort_blocks(g, 1), sort_blocks(g, 2), g.nstrip * g.nchunk,
                                       ((g.nx + 63) / 64) * I.nslice};
        for (int k = 0; k < BPRE_KINDS; ++k)
            pre[(size_t)k * (count + 1) + i + 1] = pre[(size_t)k * (count + 1) + i] + (g.n > 0 || k == BPRE_SCAN ||
                                                                                       k >= BPRE_RECON ? items[k] : 0);
        b->max_nx = std::max(b->max_nx, g.nx);
        b->lds = std::max(b->lds, sort_lds(g));
        b->lds_scatter = std::max(b->lds_scatter, scatter_lds(g));
    }
    for (int k = 0; k < BPRE_KINDS; ++k) b->tot[k] = pre[(size_t)k * (count + 1) + count];
    b->tab = (BInst*)(ws + tab_off);
    b->pre = (int*)(ws + pre_off);
    hipError_t e = hipMemcpyAsync(b->tab, tab.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->pre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) {
        for (avl_handle* q : b->h) avl_destroy(q);
        delete b;
        return report(e, "batch tables", __LINE__);
    }
    *out = b;
    return AVL_OK;
}

int avl_batch_step(avl_batch* b, int32_t nsteps, double* diag_out)
{
    if (!b) return AVL_EINVAL;
    if (nsteps < 0) return AVL_EINVAL;
    const int cur = b->h[0]->cur;
    for (avl_handle* h : b->h)
        if (!h->have_E || !h->sorted || h->cur != cur) return AVL_ESTATE;
    std::vector<int64_t> first(b->n);
    for (int i = 0; i < b->n; ++i) first[i] = b->h[i]->steps;
    int32_t s = 0;
    // a half first kick is a different launch argument: run it per instance
    if (nsteps > 0 && kick_fraction(b->h[0]) != 1.0) {
        for (avl_handle* h : b->h) {
            const hipStream_t own = h->st;
            h->st = b->st;
            const int rc = one_step(h);
            h->st = own;
            if (rc) return rc;
        }
        s = 1;
    }
    if (!b->graph_ok && s < nsteps) {
        if (!b->cap_st) AVL_TRY(hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking));
        AVL_TRY(hipStreamSynchronize(b->st));
        for (int p = 0; p < 2; ++p) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeThreadLocal);
            int rc = e == hipSuccess ? batch_launch(b, p, b->cap_st) : AVL_EDEVICE;
            hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(b->cap_st, &graph) : e;
            if (e != hipSuccess) return report(e, "hipStreamBeginCapture", __LINE__);
            if (e2 != hipSuccess) return report(e2, "hipStreamEndCapture", __LINE__);
            if (rc) return rc;
            e = hipGraphInstantiate(&b->gexec[p], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                drop_batch_graphs(b);
                return report(e, "hipGraphInstantiate", __LINE__);
            }
        }
        b->graph_ok = true;
    }
    for (; s < nsteps; ++s) {
        AVL_TRY(hipGraphLaunch(b->gexec[b->h[0]->cur], b->st));
        batch_advance(b);
        if (diag_out && ((s + 1) % kDiagCap == 0))
            for (int i = 0; i < b->n; ++i) {
                avl_handle* h = b->h[i];
                const hipStream_t own = h->st;
                h->st = b->st;
                const int rc = copy_diag(h, first[i] + s + 1 - kDiagCap, kDiagCap,
                                         diag_out + 2 * ((size_t)i * nsteps + s + 1 - kDiagCap));
                h->st = own;
                if (rc) return rc;
            }
    }
    if (diag_out) {
        const int32_t tail = nsteps % kDiagCap;
        for (int i = 0; tail && i < b->n; ++i) {
            avl_handle* h = b->h[i];
            const hipStream_t own = h->st;
            h->st = b->st;
            const int rc = copy_diag(h, first[i] + nsteps - tail, tail, diag_out + 2 * ((size_t)i * nsteps + nsteps - tail));
            h->st = own;
            if (rc) return rc;
        }
    }
    return AVL_OK;
}

avl_handle* avl_batch_instance(avl_batch* b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->h[i];
}

int avl_batch_count(const avl_batch* b) { return b ? b->n : -1; }

int avl_batch_check(avl_batch* b)
{
    if (!b) return AVL_EINVAL;
    AVL_TRY(hipStreamSynchronize(b->st));
    for (avl_handle* h : b->h) {
        const int rc = avl_check(h);
        if (rc) return rc;
    }
    return AVL_OK;
}

int avl_batch_destroy(avl_batch* b)
{
    if (!b) return AVL_EINVAL;
    drop_batch_graphs(b);
    if (b->cap_st) (void)hipStreamDestroy(b->cap_st);
    for (avl_handle* h : b->h) avl_destroy(h);
    delete b;
    return AVL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// adjoint runs (1D-1V, both storage forms)
// ---------------------------------------------------------------------------
namespace {

// Recording workspace: checkpoints (a raw copy of the marker buffer with the
// identities, and the field, every `every` steps), the states of one segment
// (FP64 positions and velocities, identities, f and D grids in the storage
// precision, the field), adjoints by marker identity, identity arrays for
// both marker buffers, small field buffers.
struct AdjLayout {
    size_t cp, cp_stride, cp_ids, cp_E, mbytes;
    size_t seg, seg_stride, st_x, st_v, st_fg, st_D, st_E;
    size_t ids[2], lam_x, lam_v, f_bar, f_by_id, Pmu, mu, diag, total;
    int nseg;
};

bool adj_layout(const avl_config* c, const Geo& g, int32_t nsteps, int32_t every, AdjLayout* A)
{
    if (nsteps < 1 || every < 1 || g.vdim != 1) return false;
    Layout L;
    make_layout(c, g, &L);
    const size_t n = (size_t)g.np, G = (size_t)g.nx * g.nv[0], nx = (size_t)g.nx;
    const size_t esz = g.prec == AVL_FP64 ? 8 : 4;
    A->mbytes = L.markers[1] - L.markers[0];
    A->nseg = (nsteps + every - 1) / every;
    size_t co = 0;
    auto ctake = [&](size_t bytes) { size_t r = co; co = align_up(co + bytes); return r; };
    ctake(A->mbytes);
    A->cp_ids = ctake(4 * n);
    A->cp_E = ctake(8 * nx);
    A->cp_stride = co;
    size_t so = 0;
    auto stake = [&](size_t bytes) { size_t r = so; so = align_up(so + bytes); return r; };
    A->st_x = stake(8 * n);
    A->st_v = stake(8 * n);
    A->st_fg = stake(esz * G);
    A->st_D = stake(esz * G);
    A->st_E = stake(8 * nx);
    A->seg_stride = so;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    A->cp = take(A->cp_stride * (size_t)A->nseg);
    A->seg = take(A->seg_stride * ((size_t)every + 1));
    A->ids[0] = take(4 * n);
    A->ids[1] = take(4 * n);
    A->lam_x = take(8 * n);
    A->lam_v = take(8 * n);
    A->f_bar = take(8 * n);
    A->f_by_id = take(8 * n);
    A->Pmu = take(8 * nx);
    A->mu = take(8 * nx);
    A->diag = take(16 * (size_t)nsteps);
    A->total = o;
    return true;
}

int* id_of(avl_handle* h, int b) { return h->g.prec == AVL_FP64 ? h->m64[b].id : h->m32[b].id; }

void set_ids(avl_handle* h, int b, int* p)
{
    if (h->g.prec == AVL_FP64) h->m64[b].id = p;
    else h->m32[b].id = p;
}

// Checkpoint: the current marker buffer as it is, its identities, the field.
int adj_checkpoint(avl_handle* h, char* C, const AdjLayout& A, bool restore)
{
    char* mk = h->ws + h->lay.markers[h->cur];
    if (!restore) {
        // the copy must hold every cell index: it is reloaded as an unsorted buffer
        const int rc = ensure_cells(h);
        if (rc) return rc;
    } else {
        h->sorted = false;
        h->cells_ok = true;
    }
    int* id = id_of(h, h->cur);
    const size_t n = (size_t)h->g.np;
    if (restore) {
        AVL_TRY(hipMemcpyAsync(mk, C, A.mbytes, hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(id, C + A.cp_ids, 4 * n, hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(h->E, C + A.cp_E, 8 * (size_t)h->g.nx, hipMemcpyDeviceToDevice, h->st));
    } else {
        AVL_TRY(hipMemcpyAsync(C, mk, A.mbytes, hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(C + A.cp_ids, id, 4 * n, hipMemcpyDeviceToDevice, h->st));
        AVL_TRY(hipMemcpyAsync(C + A.cp_E, h->E, 8 * (size_t)h->g.nx, hipMemcpyDeviceToDevice, h->st));
    }
    return AVL_OK;
}

// State record: FP64 positions and velocities of the current markers (the
// FP32 form converted exactly) in identity order, so that the reverse kernels
// read them, the weights and the adjoints at the same index, coalesced; the f
// grid and the field (its D grid is written by the reconstruction).
int adj_save(avl_handle* h, char* S, const AdjLayout& A)
{
    const Geo& g = h->g;
    const size_t n = (size_t)g.n;
    if (g.prec == AVL_FP64) {
        const M64& m = h->m64[h->cur];
        AVL_TRY(launch_by_id64(g.n, m.x, m.v, m.id, (double*)(S + A.st_x), (double*)(S + A.st_v), h->st));
    } else {
        const int rc = ensure_cells(h);
        if (rc) return rc;
        const M32& m = h->m32[h->cur];
        if (n) AVL_TRY(launch_to64(g, m, (double*)(S + A.st_x), (double*)(S + A.st_v), nullptr, h->st, m.id));
    }
    const size_t esz = g.prec == AVL_FP64 ? 8 : 4;
    AVL_TRY(hipMemcpyAsync(S + A.st_fg, h->fgrid, esz * (size_t)g.nx * g.nv[0], hipMemcpyDeviceToDevice, h->st));
    AVL_TRY(hipMemcpyAsync(S + A.st_E, h->E, 8 * (size_t)g.nx, hipMemcpyDeviceToDevice, h->st));
    return AVL_OK;
}

}  // namespace

extern "C" {

size_t avl_adjoint_workspace_bytes(const avl_config* cfg, int32_t nsteps, int32_t every)
{
    Geo g;
    if (make_geo(cfg, &g) != AVL_OK) return 0;
    AdjLayout A;
    return adj_layout(cfg, g, nsteps, every, &A) ? A.total : 0;
}

int avl_adjoint(avl_handle* h, const double* x, const double* v, const double* f, int32_t nsteps, int32_t every,
                void* rec, size_t rec_bytes, double* J_out, double* grad_f)
{
    if (!h || !rec || !J_out || !grad_f) return AVL_EINVAL;
    if (h->g.vdim != 1) return AVL_ENOTSUP;
    AdjLayout A;
    if (!adj_layout(&h->cfg, h->g, nsteps, every, &A)) return AVL_EINVAL;
    if ((uintptr_t)rec & 255) return AVL_EALIGN;
    if (rec_bytes < A.total) return AVL_ESIZE;
    if (h->timing) return AVL_ESTATE;
    const Geo& g = h->g;
    const int n = g.n;
    char* R = (char*)rec;
    double* lam_x = (double*)(R + A.lam_x);
    double* lam_v = (double*)(R + A.lam_v);
    double* f_bar = (double*)(R + A.f_bar);
    double* f_by_id = (double*)(R + A.f_by_id);
    double* Pmu = (double*)(R + A.Pmu);
    double* mu = (double*)(R + A.mu);
    double* diag = (double*)(R + A.diag);
    unsigned long long* acc = (unsigned long long*)(h->ws + h->lay.adj);
    unsigned* key = (unsigned*)(h->ws + h->lay.adj + sizeof(unsigned long long) * 2 * (size_t)h->g.nx);
    auto state = [&](int q) { return R + A.seg + A.seg_stride * (size_t)q; };
    auto ckpt = [&](int k) { return R + A.cp + A.cp_stride * (size_t)k; };
    const double dxdt2 = 2.0 * g.dx * g.dt;
    const int gp = g.prec;
    drop_graphs(h);
    for (int b = 0; b < 2; ++b) {
        set_ids(h, b, (int*)(R + A.ids[b]));
        // every slot holds a valid identity even before the first scatter fills it
        hipError_t e = hipMemsetAsync(id_of(h, b), 0, 4 * (size_t)g.np, h->st);
        if (e != hipSuccess) {
            for (int q = 0; q < 2; ++q) set_ids(h, q, nullptr);
            return report(e, "id clear", __LINE__);
        }
    }
    int rc = AVL_OK;
    auto done = [&](int r) {
        for (int b = 0; b < 2; ++b) set_ids(h, b, nullptr);
        h->rec_D = nullptr;
        return r;
    };
    // forward: load (identities = caller's order), checkpoint every `every` steps
    if (n > 0) {
        if (!x || !v || !f) return done(AVL_EINVAL);
        hipError_t e = hipMemcpyAsync(f_by_id, f, 8 * (size_t)n, hipMemcpyDeviceToDevice, h->st);
        if (e != hipSuccess) return done(report(e, "f copy", __LINE__));
    }
    if ((rc = load_markers(h, x, v, f, true))) return done(rc);
    for (int k = 0; k < A.nseg; ++k) {
        if ((rc = adj_checkpoint(h, ckpt(k), A, false))) return done(rc);
        const int s0 = k * every, s1 = std::min(nsteps, s0 + every);
        if ((rc = avl_step(h, s1 - s0, diag + 2 * (size_t)s0))) return done(rc);
    }
    // J = sum_n sum_i E_i^2 dx dt = 2 c_p dt sum_n W^n
    {
        std::vector<double> hd(2 * (size_t)nsteps);
        hipError_t e = hipMemcpyAsync(hd.data(), diag, 16 * (size_t)nsteps, hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) return done(report(e, "diag copy", __LINE__));
        double J = 0.0;
        for (int s = 0; s < nsteps; ++s) J += hd[2 * s];
        J *= 2.0 * g.cp * g.dt;
        e = hipMemcpyAsync(J_out, &J, sizeof(double), hipMemcpyHostToDevice, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) return done(report(e, "J copy", __LINE__));
    }
    // reverse sweep, one segment at a time from its checkpoint
    hipError_t e = hipMemsetAsync(lam_x, 0, 8 * (size_t)g.np, h->st);
    if (e == hipSuccess) e = hipMemsetAsync(lam_v, 0, 8 * (size_t)g.np, h->st);
    if (e == hipSuccess) e = hipMemsetAsync(f_bar, 0, 8 * (size_t)g.np, h->st);
    if (e == hipSuccess) e = launch_adj_clear(g.nx, acc, key, h->st);
    if (e != hipSuccess) return done(report(e, "adjoint clear", __LINE__));
    // mu^N = 2 dx dt E^N
    if (launch_adj_mu(g, h->E, dxdt2, acc, key, mu, h->st) != hipSuccess) return done(AVL_EDEVICE);
    const double c_full = g.qm * g.dt;
    for (int k = A.nseg - 1; k >= 0; --k) {
        const int s0 = k * every, s1 = std::min(nsteps, s0 + every);
        // restore the checkpoint, re-sort it (run bounds for the
        // reconstruction), rebuild f and D, then recompute the segment
        if ((rc = adj_checkpoint(h, ckpt(k), A, true))) return done(rc);
        h->steps = s0;
        h->kicked = s0 > 0;
        h->have_E = true;
        if ((rc = do_sort(h, false, 1.0))) return done(rc);
        if ((rc = do_recon(h, state(0) + A.st_D))) return done(rc);
        if ((rc = adj_save(h, state(0), A))) return done(rc);
        for (int q = 0; q < s1 - s0; ++q) {
            h->rec_D = state(q + 1) + A.st_D;
            if ((rc = one_step(h))) return done(rc);
            if ((rc = adj_save(h, state(q + 1), A))) return done(rc);
        }
        h->rec_D = nullptr;
        for (int q = s1 - s0 - 1; q >= 0; --q) {
            const int step = s0 + q;                       // reverse of step -> step+1
            char* S1 = state(q + 1);
            char* S0 = state(q);
            if (launch_field(g, nullptr, mu, h->rho_slices, h->rho, Pmu, h->tw, h->green, h->diag, h->ctr, 0, nullptr,
                             h->flags, h->st) != hipSuccess)
                return done(AVL_EDEVICE);
            // the states are in identity order, so the deposit reverse (state
            // step+1) and the push reverse (state step) run as one pass
            const double kick = (step == 0 && h->cfg.first_kick) ? 0.5 : 1.0;
            if (launch_adj_step_rev(g, gp, (double*)(S1 + A.st_x), (double*)(S1 + A.st_v), f_by_id, S1 + A.st_fg,
                                    S1 + A.st_D, Pmu, -1.0, (double*)(S0 + A.st_x), (double*)(S0 + A.st_E),
                                    c_full * kick, lam_x, lam_v, f_bar, acc, key, h->st) != hipSuccess)
                return done(AVL_EDEVICE);
            if (launch_adj_mu(g, (double*)(S0 + A.st_E), step >= 1 ? dxdt2 : 0.0, acc, key, mu, h->st) != hipSuccess)
                return done(AVL_EDEVICE);
        }
        if (k == 0) {
            // the initial reconstruction: weights only (the loaded positions are fixed)
            char* S0 = state(0);
            if (launch_field(g, nullptr, mu, h->rho_slices, h->rho, Pmu, h->tw, h->green, h->diag, h->ctr, 0, nullptr,
                             h->flags, h->st) != hipSuccess)
                return done(AVL_EDEVICE);
            if (launch_adj_deposit(g, gp, (double*)(S0 + A.st_x), (double*)(S0 + A.st_v), nullptr, f_by_id,
                                   S0 + A.st_fg, S0 + A.st_D, Pmu, -1.0, lam_x, lam_v, f_bar, 0, h->st) !=
                hipSuccess)
                return done(AVL_EDEVICE);
        }
    }
    e = hipMemcpyAsync(grad_f, f_bar, 8 * (size_t)n, hipMemcpyDeviceToDevice, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return done(report(e, "gradient copy", __LINE__));
    // the handle now holds a recomputed state of the first segment; its
    // field and f are current for that state
    h->have_rho = h->partials = false;
    return done(AVL_OK);
}

int avl_adjoint_deposit(avl_handle* h, const double* x, const double* v, const double* f, const void* f_grid,
                        const void* D_grid, const double* rho_bar, double* f_bar, double* lam_x, double* lam_v)
{
    if (!h) return AVL_EINVAL;
    if (h->g.vdim != 1) return AVL_ENOTSUP;
    const Geo& g = h->g;
    if (!f_grid || !D_grid || !rho_bar) return AVL_EINVAL;
    if (g.n > 0 && (!x || !v || !f || !f_bar)) return AVL_EINVAL;
    if ((lam_x == nullptr) != (lam_v == nullptr)) return AVL_EINVAL;
    const uintptr_t gal = g.prec == AVL_FP64 ? 7 : 3;
    if (((uintptr_t)x | (uintptr_t)v | (uintptr_t)f | (uintptr_t)rho_bar | (uintptr_t)f_bar | (uintptr_t)lam_x |
         (uintptr_t)lam_v) & 7)
        return AVL_EALIGN;
    if (((uintptr_t)f_grid | (uintptr_t)D_grid) & gal) return AVL_EALIGN;
    if (h->timing) return AVL_ESTATE;
    AVL_TRY(launch_fill_f64(f_bar, g.n, 0.0, h->st));
    if (lam_x) {
        AVL_TRY(launch_fill_f64(lam_x, g.n, 0.0, h->st));
        AVL_TRY(launch_fill_f64(lam_v, g.n, 0.0, h->st));
    }
    AVL_TRY(launch_adj_deposit(g, g.prec, x, v, nullptr, f, f_grid, D_grid, rho_bar, 1.0, lam_x, lam_v, f_bar,
                               lam_x ? 1 : 0, h->st));
    return AVL_OK;
}

int avl_adjoint_push(avl_handle* h, const double* x, const double* E, double kick, const double* lam_x_in,
                     const double* lam_v_in, double* lam_x, double* lam_v, double* E_bar)
{
    if (!h) return AVL_EINVAL;
    if (h->g.vdim != 1) return AVL_ENOTSUP;
    const Geo& g = h->g;
    if (!E || !E_bar || !std::isfinite(kick)) return AVL_EINVAL;
    if (g.n > 0 && (!x || !lam_x_in || !lam_v_in || !lam_x || !lam_v)) return AVL_EINVAL;
    if (((uintptr_t)x | (uintptr_t)E | (uintptr_t)lam_x_in | (uintptr_t)lam_v_in | (uintptr_t)lam_x |
         (uintptr_t)lam_v | (uintptr_t)E_bar) & 7)
        return AVL_EALIGN;
    if (h->timing) return AVL_ESTATE;
    unsigned long long* acc = (unsigned long long*)(h->ws + h->lay.adj);
    unsigned* key = (unsigned*)(h->ws + h->lay.adj + sizeof(unsigned long long) * 2 * (size_t)g.nx);
    AVL_TRY(launch_adj_clear(g.nx, acc, key, h->st));
    AVL_TRY(launch_adj_push(g, x, nullptr, E, g.qm * g.dt * kick, lam_x_in, lam_v_in, lam_x, lam_v, acc, key, h->st));
    AVL_TRY(launch_adj_mu(g, nullptr, 0.0, acc, key, E_bar, h->st));
    return AVL_OK;
}

int avl_adjoint_field(avl_handle* h, const double* mu, double* rho_bar)
{
    if (!h || !mu || !rho_bar) return AVL_EINVAL;
    if (((uintptr_t)mu | (uintptr_t)rho_bar) & 7) return AVL_EALIGN;
    if (mu == rho_bar) return AVL_EINVAL;
    if (h->timing) return AVL_ESTATE;
    const Geo& g = h->g;
    AVL_TRY(launch_field(g, nullptr, mu, h->rho_slices, h->rho, rho_bar, h->tw, h->green, h->diag, h->ctr, 0, nullptr,
                         h->flags, h->st));
    AVL_TRY(launch_scale_f64(rho_bar, g.nx, -1.0, h->st));
    return AVL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Several species in one self-consistent field
// ---------------------------------------------------------------------------

struct avl_multi {
    std::vector<avl_handle*> hs;
    Species* tab;          // device table, in the caller's workspace
    double* rho_total;     // device, nx doubles
};

namespace {

size_t multi_layout(int32_t n, int32_t nx, size_t* tab_off, size_t* rho_off)
{
    size_t off = 0;
    *tab_off = off;
    off = align_up(off + sizeof(Species) * (size_t)n);
    *rho_off = off;
    off = align_up(off + sizeof(double) * (size_t)nx);
    return off;
}

// Total rho from the species' rho (from_rho) or their fresh slices, the
// field from it into species 0, copied to the others.
int multi_field(avl_multi* m, bool from_rho, bool diag)
{
    avl_handle* h0 = m->hs[0];
    const int ns = (int)m->hs.size();
    AVL_TRY(launch_species_rho(m->tab, ns, h0->g.nx, from_rho ? 1 : 0, m->rho_total, h0->st));
    AVL_TRY(launch_field(h0->g, nullptr, m->rho_total, h0->rho_slices, h0->rho, h0->E, h0->tw, h0->green, h0->diag,
                         h0->ctr, diag ? 1 : 0, nullptr, h0->flags, h0->st));
    AVL_TRY(launch_broadcast_E(m->tab, ns, h0->g.nx, h0->st));
    for (avl_handle* h : m->hs) h->have_rho = h->have_E = true;
    return AVL_OK;
}

}  // namespace

extern "C" {

size_t avl_multi_workspace_bytes(int32_t nspecies, int32_t nx)
{
    if (nspecies < 1 || nspecies > 64 || nx < 8 || nx > kMaxNx) return 0;
    size_t a, b;
    return multi_layout(nspecies, nx, &a, &b);
}

int avl_multi_init(avl_handle* const* hs, int32_t n, void* workspace, size_t bytes, avl_multi** out)
{
    if (!out) return AVL_EINVAL;
    *out = nullptr;
    if (!hs || n < 1 || n > 64 || !workspace) return AVL_EINVAL;
    for (int32_t s = 0; s < n; ++s) {
        if (!hs[s]) return AVL_EINVAL;
        for (int32_t r = 0; r < s; ++r)
            if (hs[r] == hs[s]) return AVL_EINVAL;
    }
    const avl_handle* h0 = hs[0];
    for (int32_t s = 1; s < n; ++s) {
        const avl_config &a = h0->cfg, &b = hs[s]->cfg;
        // one x grid, one field, one time step, one stream
        if (a.nx != b.nx || a.L != b.L || a.c_p != b.c_p || a.dt != b.dt || a.first_kick != b.first_kick)
            return AVL_EINVAL;
        if (hs[s]->st != h0->st) return AVL_EINVAL;
    }
    for (int32_t s = 0; s < n; ++s)
        if (!hs[s]->have_rho || !hs[s]->sorted) return AVL_ESTATE;
    if ((uintptr_t)workspace % kAlign) return AVL_EALIGN;
    size_t tab_off, rho_off;
    if (bytes < multi_layout(n, h0->g.nx, &tab_off, &rho_off)) return AVL_ESIZE;
    avl_multi* m = new (std::nothrow) avl_multi;
    if (!m) return AVL_EDEVICE;
    m->hs.assign(hs, hs + n);
    m->tab = (Species*)((char*)workspace + tab_off);
    m->rho_total = (double*)((char*)workspace + rho_off);
    std::vector<Species> tab(n);
    for (int32_t s = 0; s < n; ++s) {
        avl_handle* h = hs[s];
        tab[s] = Species{h->rho_slices, field_slices(h->g), h->g.q_vol, h->rho, h->E};
    }
    hipError_t e = hipMemcpyAsync(m->tab, tab.data(), sizeof(Species) * n, hipMemcpyHostToDevice, h0->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h0->st);
    if (e != hipSuccess) {
        delete m;
        return report(e, "species table upload", __LINE__);
    }
    // the initial field from the total charge density
    int rc = multi_field(m, true, false);
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return AVL_OK;
}

int avl_multi_step(avl_multi* m, int32_t nsteps, double* diag_out)
{
    if (!m) return AVL_EINVAL;
    if (nsteps < 0) return AVL_EINVAL;
    for (avl_handle* h : m->hs)
        if (!h->have_E || !h->sorted) return AVL_ESTATE;
    avl_handle* h0 = m->hs[0];
    const int64_t first = h0->steps;
    for (int32_t step = 0; step < nsteps; ++step) {
        int rc;
        for (avl_handle* h : m->hs)
            if ((rc = do_sort(h, true, kick_fraction(h)))) return rc;
        for (avl_handle* h : m->hs) {
            if ((rc = do_recon(h, nullptr))) return rc;
            AVL_TRY(launch_rho_slices(h->g, h->rho_part, h->rho_slices, h->st));
        }
        if ((rc = multi_field(m, false, true))) return rc;
        for (avl_handle* h : m->hs) h->steps += 1;
        if (diag_out && ((step + 1) % kDiagCap == 0)) {
            if ((rc = copy_diag(h0, first + step + 1 - kDiagCap, kDiagCap, diag_out + 2 * (step + 1 - kDiagCap))))
                return rc;
        }
    }
    if (diag_out) {
        const int32_t tail = nsteps % kDiagCap;
        if (tail) return copy_diag(h0, first + nsteps - tail, tail, diag_out + 2 * (nsteps - tail));
    }
    return AVL_OK;
}

int avl_multi_destroy(avl_multi* m)
{
    if (!m) return AVL_EINVAL;
    delete m;
    return AVL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Reconstruction without allocation (avl_reconstruct_noalloc).
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid it) get the load, sort and
// reconstruction of avl_init + avl_reconstruct with every scratch buffer in
// one file-scope device array.  In host code `scratch` only names the array:
// its device address comes from hipGetSymbolAddress, looked up once per
// device with that device current, and only that address is ever handed to
// kernels.  Every call on a GPU shares the array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[AVL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there); null on failure.
void* scratch_address()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

__global__ void k_fill_int(int* __restrict__ p, int n, int value)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = value;
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

hipError_t fill_int(int* p, size_t n, int value, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_int, dim3(blocks), dim3(256), 0, st, p, (int)n, value);
    return hipGetLastError();
}

hipError_t copy_f64(const double* src, double* dst, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy_f64, dim3(blocks), dim3(256), 0, st, src, dst, (int)n);
    return hipGetLastError();
}

}  // namespace

extern "C" int avl_reconstruct_noalloc(const avl_config* cfg, void* stream, const double* x, const double* v,
                                       const double* f, void* f_out, void* D_out)
{
    Geo g;
    int rc = make_geo(cfg, &g);
    if (rc) return rc;
    if (!f_out) return AVL_EINVAL;
    if (g.n > 0 && (!x || !v || !f)) return AVL_EINVAL;
    if (((uintptr_t)x | (uintptr_t)v | (uintptr_t)f) & 7) return AVL_EALIGN;
    if (((uintptr_t)f_out | (uintptr_t)D_out) & 7) return AVL_EALIGN;
    // the slice of the handle layout this call needs: two marker buffers,
    // counts, offsets, per-scan-tile totals, the rho partials and the flags
    const size_t np = (size_t)g.np;
    const size_t mbytes = (g.prec == AVL_FP64 ? sizeof(double) * np * (2 + g.vdim) : 4 * np * (3 + g.vdim)) +
                          64 * (3 + g.vdim);
    const size_t nbt = (size_t)g.nb + 1;
    const size_t ntiles = (nbt + kScanTile - 1) / kScanTile;
    const size_t tstride = ntiles + 64;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const size_t o_m0 = take(mbytes), o_m1 = take(mbytes);
    const size_t o_counts = take(sizeof(int) * nbt), o_offsets = take(sizeof(int) * (nbt + 1));
    const size_t o_tsum = take(sizeof(int) * 2 * tstride);
    const size_t o_rho = take(sizeof(double) * (size_t)std::max(1, g.nchunk) * g.nx);
    const size_t o_flags = take(sizeof(int));
    if (off > (size_t)AVL_NOALLOC_SCRATCH_BYTES) return AVL_ESIZE;
    char* base = (char*)scratch_address();
    if (!base) return AVL_EDEVICE;
    const hipStream_t st = (hipStream_t)stream;
    // launch shapes as avl_init sets them (device attributes and occupancy only)
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) != hipSuccess) return AVL_EDEVICE;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || lds <= 0)
            if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
        set_lds_limit(lds);
        fit_lds(&g, lds);
        sort_launch_shapes(g);
    }
    M64 m64[2];
    M32 m32[2];
    for (int b = 0; b < 2; ++b) {
        char* p = base + (b ? o_m1 : o_m0);
        if (g.prec == AVL_FP64) {
            double* d = reinterpret_cast<double*>(p);
            m64[b] = M64{d, d + np, d + np * (1 + g.vdim), nullptr};
        } else {
            int* c = reinterpret_cast<int*>(p);
            m32[b] = M32{c, reinterpret_cast<float*>(c + np), reinterpret_cast<float*>(c + 2 * np),
                         reinterpret_cast<float*>(c + np * (2 + g.vdim)), nullptr};
        }
    }
    int* counts = (int*)(base + o_counts);
    int* offsets = (int*)(base + o_offsets);
    int* tsum = (int*)(base + o_tsum);
    double* rho_part = (double*)(base + o_rho);
    int* flags = (int*)(base + o_flags);
    // the array keeps the previous call's contents: clear what the passes
    // accumulate into (counts, both halves of the tile totals, flags) and set
    // the end offset, all with kernels (no memset or host copy)
    AVL_TRY(fill_int(counts, nbt, 0, st));
    AVL_TRY(fill_int(tsum, 2 * tstride, 0, st));
    AVL_TRY(fill_int(flags, 1, 0, st));
    AVL_TRY(fill_int(offsets + nbt, 1, g.n, st));
    const size_t n = (size_t)g.n;
    if (g.prec == AVL_FP64) {
        AVL_TRY(copy_f64(x, m64[0].x, n, st));
        for (int d = 0; d < g.vdim; ++d) AVL_TRY(copy_f64(v + (size_t)d * n, m64[0].v + (size_t)d * np, n, st));
        AVL_TRY(copy_f64(f, m64[0].f, n, st));
    } else {
        AVL_TRY(launch_to32(g, x, v, f, m32[0], flags, st));
    }
    void* src = g.prec == AVL_FP64 ? (void*)&m64[0] : (void*)&m32[0];
    void* dst = g.prec == AVL_FP64 ? (void*)&m64[1] : (void*)&m32[1];
    for (int phase = 0; phase < 3; ++phase)
        AVL_TRY(launch_sort(g, src, dst, nullptr, nullptr, g.dt, g.bscale, counts, offsets, tsum, tsum + tstride,
                            flags, false, st, phase, nullptr, nullptr, nullptr));
    if (g.vdim == 1) AVL_TRY(launch_recon(g, dst, offsets, f_out, D_out, rho_part, st));
    else AVL_TRY(launch_recon3(g, dst, offsets, f_out, D_out, rho_part, nullptr, st));
    return AVL_OK;
}
