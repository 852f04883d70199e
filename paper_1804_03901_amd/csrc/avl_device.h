// Device-side definitions shared by the libavl kernels (gfx950).
//
// Phase-space bookkeeping used throughout:
//  * A marker at x has the dual coordinate s = x/dx - 1/2: the integer part
//    i0 = floor(s) is the x cell whose centre is the marker's left cloud
//    neighbour and a = s - i0 in [0,1) is the cloud-in-cell weight of the right
//    neighbour (Sec. 2, Fig. "interpolation"; centres as in Fig. "phasespace").
//    The same holds per velocity component with t = (v - vmin)/dv - 1/2,
//    j0 = floor(t), b = t - j0.
//  * Markers are sorted by "bucket": the dual cell (i0 mod nx, j0+1 per velocity
//    component), flattened velocity-major with nv[d]+1 dual rows per component
//    (j0 ranges over -1..nv-1 for clouds that still touch the grid).  Clouds
//    that miss the velocity grid entirely go to one overflow bucket (index nb),
//    which the reconstruction ignores.  Bucket rows therefore have nx entries.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace avl {

enum : int { FLAG_NONFINITE = 1, FLAG_SLOT = 2, FLAG_RANGE = 4 };

constexpr int kWave = 64;
constexpr int kSortThreads = 256;
constexpr int kSortMPT = 8;                               // markers per thread, scatter pass
constexpr int kSortTile = kSortThreads * kSortMPT;
constexpr int kCountMPT = 16;                             // markers per thread, count pass, FP32 form
constexpr int kCountMPT64 = 12;                           // the same for the FP64 path (more registers a marker)
constexpr int kCountTile = kSortThreads * kCountMPT;      // the larger count tile (window sizing)
template <int PREC> constexpr int count_mpt() { return PREC ? kCountMPT : kCountMPT64; }
constexpr int count_tile_size(int prec) { return kSortThreads * (prec ? kCountMPT : kCountMPT64); }
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kReconCols = kWave - 1;                     // target columns per reconstruct wave
constexpr int kDiagCap = 4096;                            // per-step diagnostics ring
constexpr int kFieldThreads = 1024;                      // threads of a field-solve block
constexpr int kMaxFieldSlices = 64;                       // chunk slices of the rho reduction
constexpr int kMaxNx = 4096;
constexpr int kDiagThreads = 256;                        // columns per diagnostics block
constexpr int kDiagBlocks = 1024;                        // target blocks of the diagnostics pass

struct Geo {
    int vdim, prec;
    int nx, lognx;
    int nv[3];
    int nrow;            // number of bucket rows: prod(nv[d] + 1)
    int nb;              // in-range buckets nrow*nx; bucket nb collects the rest
    int n;               // markers
    int np;              // stride between velocity components in marker storage (n padded to 64)
    int rc;              // target velocity rows per reconstruct chunk (1D-1V)
    int nchunk, nstrip;  // reconstruct chunks along v and column strips along x
    int hist_bins;       // LDS histogram bins per sort block
    int sbins;           // LDS histogram bins of the step's scatter (FP32 1D-1V), at most hist_bins
    int cap;             // markers staged in LDS per reconstruct wave
    int jpad, jrange;    // FP32 1D-3V: x-velocity dual index stored with offset jpad, range jrange
    int kahan;           // FP32 form: compensated FP32 accumulation instead of FP64 accumulators
    int sblocks;         // blocks of the tiled scatter (FP32 1D-1V): the resident capacity; 0 = a tile per block
    int sblocks_step;    // blocks of the step's scatter (FP32 1D-1V): its resident capacity
    int cblocks;         // blocks of the count pass: its resident capacity; 0 = a tile per block
    int sort_cap;        // at most this many resident blocks per CU in the tiled sort passes (0: no limit)
    int rform;           // FP32 1D-1V reconstruction rows: 0 chosen from the shape, 1 dense, 2 sparse
    int magnetic;        // 1D-3V FP64 with a background magnetic field: Boris push
    double B[3];         // background magnetic field
    double L, inv_L, dx, inv_dx;
    double vmin[3], dv[3], inv_dv[3];
    double dt, qm, cp;
    double q_vol;        // q * prod(dv): scale from sum_j f to rho
    float bscale;        // FP32 form: q/m * dt / dv[0] (times the kick fraction)
    float gam;           // FP32 form: dv[0] * dt / dx (drift in x cells per unit b)
    float c0f;           // FP32 form: vmin[0]/dv[0] + 1/2
};

struct M64 {             // plain FP64 marker arrays
    double* x;
    double* v;           // component d of marker l at v[d*np + l]
    double* f;
    int* id;             // optional marker identities carried through the sort (adjoint runs), else null
};

struct M32 {             // FP32 form: dual cell index + offsets
    int* cell;
    float* a;
    float* b;            // component d of marker l at b[d*np + l]
    float* f;
    int* id;             // optional marker identities carried through the sort (adjoint runs), else null
};

// Drift table for the FP32 form, one entry per dual row j' = j0+1 in [0, nv]:
// the x shift in cells of a marker at b = 0, split into an integer and a
// fractional part computed once in FP64 on the host.
struct RowShift {
    int whole;
    float frac;
};

// One species of a multi-species step, as the shared-field kernels see it:
// its rho slices (unscaled sums of f over chunk ranges), their count, its
// scale q prod(dv), and its rho and E buffers.
struct Species {
    const double* rho_slices;
    int nslice;
    double q_vol;
    double* rho;
    double* E;
};

// One 1D-1V instance of a batch, as the batched kernels see it: its geometry
// and the buffers of its own workspace slice (the same layout a single handle
// uses).  Markers alternate between two buffers; the parity selects them.
struct BInst {
    Geo g;
    M64 m64[2];
    M32 m32[2];
    double* E;                 // the field (read by the push, written by the solve)
    const RowShift* rows;
    int* counts;
    int* offsets[2];           // run offsets of the order of marker buffer p
    int* tfirst[2];            // bucket of every 2048th position of that order (implied FP32 cells)
    int* tsum[2];              // per-scan-tile totals, by buffer parity
    void* fgrid;
    double* rho_part;
    double* rho_slices;
    double* rho;
    const double2* tw;
    const double* green;
    double* diag;
    long long* ctr;
    int* flags;
    double dtk;                // full-step kick
    float bk;
    int nslice;                // chunk slices of the rho reduction
};

// Work-item prefixes of a batch: instance i owns items [pre[i], pre[i+1]) of
// a batched launch.  Returns the instance of item b (pre has ninst+1 entries).
__device__ __forceinline__ int find_inst(const int* __restrict__ pre, int ninst, int b)
{
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

enum : int { BPRE_COUNT = 0, BPRE_SCAN = 1, BPRE_SCATTER = 2, BPRE_RECON = 3, BPRE_RHO = 4, BPRE_KINDS = 5 };

// Dynamic LDS a block may opt into on the current device (set at load time).
int lds_limit();

// Raise a kernel's dynamic-LDS allowance to `bytes` if it is not already that
// high (`granted` caches what was set for this kernel).
inline hipError_t ensure_lds(const void* fn, size_t bytes, int& granted)
{
    if ((int)bytes <= granted || bytes <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) granted = (int)bytes;
    return e;
}

__device__ __forceinline__ int wrap_pow2(int i, int nx) { return i & (nx - 1); }

// Raw buffer descriptor (gfx9 family, 32-bit raw data) over `bytes` bytes at
// p: buffer loads past the end return zero instead of touching memory, so
// loads of a ragged tail need no branches.  num_records is a 32-bit byte
// count; callers keep each descriptor's range below 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, size_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                             (int)(unsigned)min(bytes, (size_t)0xffffffffu), 0x00020000);
}

// Bucket of an FP64 marker and its in-cell offsets.  Returns g.nb when the
// cloud misses the velocity grid (or a coordinate is not finite).
template <int VD>
__device__ __forceinline__ int locate64(const Geo& g, double x, const double* vv,
                                        int& ix, int* jp, double& a, double* b)
{
    double s = x * g.inv_dx - 0.5;
    bool ok = (s >= -1.0) && (s < (double)g.nx);
    double sc = ok ? s : 0.0;
    double fs = floor(sc);
    a = sc - fs;
    ix = wrap_pow2((int)fs, g.nx);
    int row = 0;
#pragma unroll
    for (int d = VD - 1; d >= 0; --d) {
        double t = (vv[d] - g.vmin[d]) * g.inv_dv[d] - 0.5;
        bool okd = (t >= -1.0) && (t < (double)g.nv[d]);
        double tc = okd ? t : 0.0;
        double ft = floor(tc);
        b[d] = tc - ft;
        jp[d] = (int)ft + 1;
        ok = ok && okd;
        row = row * (g.nv[d] + 1) + jp[d];
    }
    return ok ? row * g.nx + ix : g.nb;
}

// Gather + kick + drift of one FP64 marker.  Without a magnetic field only
// the x velocity changes.  With one (1D-3V), the velocity update is the Boris
// scheme: half an electric kick h = (q/m) E dtk / 2, a rotation about B by
// t = (q/m) B dtk / 2 (u' = u + u x t, u+ = u + (2 / (1 + |t|^2)) u' x t), and
// the second half kick; the rotation keeps |v| and turns it by 2 atan(|t|).
template <int VD>
__device__ __forceinline__ void push64(const Geo& g, const double* sE, double dtk, double& x, double* v)
{
    double s = x * g.inv_dx - 0.5;
    double fs = floor(s);
    double a = s - fs;
    int ia = wrap_pow2((int)fs, g.nx);
    int ib = wrap_pow2(ia + 1, g.nx);
    double El = (1.0 - a) * sE[ia] + a * sE[ib];
    if (VD == 3 && g.magnetic) {
        const double h = 0.5 * g.qm * El * dtk;
        const double c = 0.5 * g.qm * dtk;
        const double tx = c * g.B[0], ty = c * g.B[1], tz = c * g.B[2];
        const double sc = 2.0 / (1.0 + ((tx * tx + ty * ty) + tz * tz));
        const double ux = v[0] + h, uy = v[1], uz = v[2];
        const double px = ux + (uy * tz - uz * ty);
        const double py = uy + (uz * tx - ux * tz);
        const double pz = uz + (ux * ty - uy * tx);
        v[0] = (ux + sc * (py * tz - pz * ty)) + h;
        v[1] = uy + sc * (pz * tx - px * tz);
        v[2] = uz + sc * (px * ty - py * tx);
    } else {
        v[0] = v[0] + g.qm * El * dtk;
    }
    const double vx = v[0];
    double xn = x + vx * g.dt;
    xn = xn - g.L * floor(xn * g.inv_L);
    if (xn >= g.L) xn -= g.L;
    if (xn < 0.0) xn += g.L;
    x = xn;
}

// FP32 form: bucket of a stored cell index.  1D-1V stores cell = j'*nx + i0
// with j' = j0+1 unbounded; 1D-3V stores ((jz'*(nvy+1) + jy')*jrange + jx' +
// jpad)*nx + i0 so that x-velocity rows beyond the grid stay representable.
template <int VD>
__device__ __forceinline__ int bucket32(const Geo& g, int cell)
{
    if (VD == 1) return (cell >= 0 && cell < g.nb) ? cell : g.nb;
    int ix = cell & (g.nx - 1);
    int r = cell >> g.lognx;
    // jrange is a power of two (a wave-uniform shift, no integer division)
    int jx = (r & (g.jrange - 1)) - g.jpad;
    int yz = r >> __builtin_ctz(g.jrange);
    // a (vy, vz) row index past the last plane has no bucket either
    if (cell < 0 || jx < 0 || jx > g.nv[0] || yz >= (g.nv[1] + 1) * (g.nv[2] + 1)) return g.nb;
    return (yz * (g.nv[0] + 1) + jx) * g.nx + ix;
}

// Gather + kick + drift of one FP32-form marker.  Velocity moves in units of
// dv (b carries into the dual row), position in units of dx (a carries into
// the column, with periodic wrap); the large per-row part of the x shift comes
// from the FP64-built table so no absolute coordinate is ever held in FP32.
// sE[i] holds the kick in units of dv at cell centre i, e_i = (q/m) E_i dt /
// dv (times the kick fraction), and its forward difference e_{i+1} - e_i
// (periodic), so the linear gather is one LDS read and one multiply-add.
// The push of push32 in three parts, so that a pass needing only the new
// bucket can take them over a group of markers at once.  kick32: the gather
// and the velocity update, giving the column ix, the new x-velocity row jx
// (unbounded), the (vy, vz) plane index and the offset bn in [0, 1).
template <int VD>
__device__ __forceinline__ void kick32(const Geo& g, const float2* sE, int cell, float a, float b,
                                       int& ix, int& jx, int& rest, float& bn)
{
    ix = cell & (g.nx - 1);
    const int r = cell >> g.lognx;
    if (VD == 1) { jx = r; rest = 0; }
    else { jx = (r & (g.jrange - 1)) - g.jpad; rest = r >> __builtin_ctz(g.jrange); }
    const float2 e = sE[ix];
    bn = b + (e.x + a * e.y);
    const float fl = floorf(bn);
    jx += (int)fl;
    bn -= fl;
    if (bn >= 1.0f) { bn -= 1.0f; jx += 1; }
}

// The x shift of row jx in FP32 (rows beyond the FP64-built table).
__device__ __forceinline__ void row_shift32(const Geo& g, int jx, int& whole, float& frac)
{
    const float P = ((float)(jx - 1) + g.c0f) * g.gam;
    const float Pf = floorf(P);
    whole = (int)Pf;
    frac = P - Pf;
}

// The drift: the new column from a, the row's shift and bn; a becomes the new
// offset in [0, 1).
__device__ __forceinline__ int drift32(const Geo& g, int ix, float& a, float bn, int whole, float frac)
{
    float an = a + frac + bn * g.gam;
    float ca = floorf(an);
    an -= ca;
    if (an >= 1.0f) { an -= 1.0f; ca += 1.0f; }
    a = an;
    return (ix + whole + (int)ca) & (g.nx - 1);
}

// The largest x-velocity row of a 1D-1V cell index: rows up to it keep
// cell = row * nx + column inside 32 bits; rows beyond are clamped to it and
// flagged.
__device__ __forceinline__ int row_limit32(const Geo& g) { return 1 << (30 - g.lognx); }

// Gather + kick + drift of one FP32-form marker.  Velocity moves in units of
// dv (b carries into the dual row), position in units of dx (a carries into
// the column, with periodic wrap); the large per-row part of the x shift comes
// from the FP64-built table so no absolute coordinate is ever held in FP32.
// sE[i] holds the kick in units of dv at cell centre i, e_i = (q/m) E_i dt /
// dv (times the kick fraction), and its forward difference e_{i+1} - e_i
// (periodic), so the linear gather is one LDS read and one multiply-add.
template <int VD>
__device__ __forceinline__ void push32(const Geo& g, const float2* sE, const RowShift* rows,
                                       int& cell, float& a, float& b, int& flags)
{
    int ix, jx, rest;
    float bn;
    kick32<VD>(g, sE, cell, a, b, ix, jx, rest, bn);
    // rows inside the table take its FP64-built shift, rows beyond it the FP32
    // formula; both are formed and one selected, without a branch
    const bool in_table = jx >= 0 && jx <= g.nv[0];
    const RowShift rs = rows[min(max(jx, 0), g.nv[0])];
    int wf;
    float ff;
    row_shift32(g, jx, wf, ff);
    const int whole = in_table ? rs.whole : wf;
    const float frac = in_table ? rs.frac : ff;
    float an = a;
    ix = drift32(g, ix, an, bn, whole, frac);
    if (VD == 1) {
        const int lim = row_limit32(g);
        const int jc = min(max(jx, -lim), lim);
        if (jc != jx) flags |= FLAG_RANGE;
        cell = (int)((unsigned)jc << g.lognx) + ix;
    } else {
        const int jj = jx + g.jpad;
        const int jc = min(max(jj, 0), g.jrange - 1);
        if (jc != jj) flags |= FLAG_RANGE;
        cell = (rest * g.jrange + jc) * g.nx + ix;
    }
    // an and bn lie in [0, 1) unless a NaN or infinity came in
    if (!(an + bn == an + bn)) flags |= FLAG_NONFINITE;
    a = an;
    b = bn;
}

// The new buckets of K 1D-1V FP32-form markers after push32, without the
// markers themselves or the flags (for a pass whose markers are pushed again,
// with the same field, by a pass that raises them).  Every marker reads the
// table's row shift; the FP32 formula is formed only in a branch, which a
// wave enters when one of its markers lies beyond the table.  The bucket is
// bucket32 of push32's clamped cell index, bit for bit.
template <int K>
__device__ __forceinline__ void push32_buckets(const Geo& g, const float2* sE, const RowShift* rows,
                                               const int* cell, const float* a, const float* b, int* bkt)
{
    int ix[K], jx[K], whole[K];
    float bn[K], frac[K];
    bool beyond = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int rest;
        kick32<1>(g, sE, cell[k], a[k], b[k], ix[k], jx[k], rest, bn[k]);
        const RowShift rs = rows[min(max(jx[k], 0), g.nv[0])];
        whole[k] = rs.whole;
        frac[k] = rs.frac;
        beyond |= !(jx[k] >= 0 && jx[k] <= g.nv[0]);
    }
    if (beyond) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (!(jx[k] >= 0 && jx[k] <= g.nv[0])) row_shift32(g, jx[k], whole[k], frac[k]);
    }
    const int lim = row_limit32(g);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float an = a[k];
        const int nix = drift32(g, ix[k], an, bn[k], whole[k], frac[k]);
        // rows below 0 and from nrow on have no bucket; the lower clamp of
        // push32 cannot bring a row into range, the upper one can
        const int jc = min(jx[k], lim);
        bkt[k] = (unsigned)jc < (unsigned)g.nrow ? (int)((unsigned)jc << g.lognx) + nix : g.nb;
    }
}

// ---------------------------------------------------------------------------
// Order-independent sums over a run of markers.
//
// The markers of one cell arrive in an order set by the sort's integer
// atomics, which varies from run to run.  To make every reconstruction sum a
// function of the run's multiset alone, each term is rounded down onto a grid
// of spacing q = 2^e, chosen per run from an order-free bound (the run length
// times the largest magnitude of its terms), and the grid points are added
// exactly:
//  * the accumulator starts at C = 3 * 2^51 * q; every value within 2^51 q of
//    C is an FP64 number whose spacing is exactly q;
//  * with the FP64 rounding mode set toward -infinity, acc + t (or a fused
//    acc + x*y) then yields C + (m + floor(t/q)) q exactly;
//  * so acc - C = q * sum floor(t/q) over the run, in any order.
// The error is below q per term, i.e. below len * 2^-51 of the bound.  Code
// between fixsum_round_down() and fixsum_round_nearest() must only add terms
// to such accumulators; the values that cross either switch go through
// fixsum_pin(), which keeps the compiler from moving their arithmetic across
// it.  Where a loop also needs ordinary FP64 arithmetic (locating an FP64
// marker), fixsum_floor() rounds a term onto the grid explicitly instead.
// ---------------------------------------------------------------------------
struct FixGrid {
    double q;       // grid spacing 2^e
    double inv_q;   // 2^-e
    double C;       // accumulator origin 3 * 2^51 * q
};

// Power of two 2^e as an FP64 number, for e in the normal range.
__device__ __forceinline__ double fix_pow2(int e) { return __longlong_as_double((long long)(e + 1023) << 52); }

// Grid exponent for len terms of magnitude below 2^(emax + 1).  It is kept
// where q, 1/q and C are all normal numbers (a coarser grid for terms below
// 2^-900 still bounds them).
__device__ __forceinline__ int fix_exponent(int emax, int len)
{
    const int lg = len > 1 ? 32 - __builtin_clz((unsigned)(len - 1)) : 0;     // ceil(log2(len))
    return min(max(emax + 1 + lg - 51, -960), 960);
}

// The accumulator origin C = 3 * 2^51 * q alone (all the rounding-mode path needs).
__device__ __forceinline__ double fix_origin(int emax, int len) { return 3.0 * fix_pow2(fix_exponent(emax, len) + 51); }

__device__ __forceinline__ FixGrid fix_grid(int emax, int len)
{
    const int e = fix_exponent(emax, len);
    FixGrid gr;
    gr.q = fix_pow2(e);
    gr.inv_q = fix_pow2(-e);
    gr.C = 3.0 * fix_pow2(e + 51);
    return gr;
}

// floor(log2 |x|) bounds from the raw bits: |x| < 2^(e + 1) with e the
// returned value (denormals and zero give the smallest normal exponent - 1).
// For the largest e over many values, take the largest fix_key (the
// magnitude's bits, which order like the magnitudes) and convert it once.
__device__ __forceinline__ unsigned fix_key(float x) { return __float_as_uint(x) & 0x7fffffffu; }
__device__ __forceinline__ unsigned fix_key(double x) { return (unsigned)(__double_as_longlong(x) >> 32) & 0x7fffffffu; }
__device__ __forceinline__ int fix_exp_of_key(unsigned k, float) { return (int)(k >> 23) - 127; }
__device__ __forceinline__ int fix_exp_of_key(unsigned k, double) { return (int)(k >> 20) - 1023; }
template <typename T> __device__ __forceinline__ int fix_exp_bits(T x) { return fix_exp_of_key(fix_key(x), x); }

// Issue priority from progress: a wave that has done `done` of its `total`
// units of work (rows, tiles) takes priority 3 in its first quarter down to 0
// in its last.  A compute unit's waves then issue in the order of how far
// behind they are, so the ones that fell behind catch up and fewer are still
// running at the end of a launch, when the memory system is no longer
// saturated.  Priority only orders issue; results do not depend on it.
__device__ __forceinline__ void prio_by_progress(int done, int total)
{
    const int pr = 3 - min(3, (4 * done) / max(total, 1));
    if (pr >= 3) __builtin_amdgcn_s_setprio(3);
    else if (pr == 2) __builtin_amdgcn_s_setprio(2);
    else if (pr == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ void fixsum_pin(double& v) { asm volatile("" : "+v"(v)); }

// FP64 rounding mode (MODE register, FP_ROUND bits 3:2): toward -infinity, and
// back to the default nearest-even.  The FP32 rounding bits are left alone.
// Written as inline assembly on purpose: the compiler's mode-register pass
// treats a mode it knows to be non-default as something to undo, and inserts
// a switch back to nearest-even in front of instructions such as v_mul_f64,
// which would silently end the region.  The switch is ordered against the
// accumulators by fixsum_pin() (volatile asm statements keep their order); the
// s_nop gives the new mode time to reach the vector pipeline.
__device__ __forceinline__ void fixsum_round_down() { asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\ts_nop 3"); }
__device__ __forceinline__ void fixsum_round_nearest() { asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0\n\ts_nop 3"); }

// floor(t / q) * q added to an accumulator that holds a multiple of q (used
// in the default rounding mode; the multiplication by 2^-e is exact).
__device__ __forceinline__ double fixsum_floor(const FixGrid& gr, double t) { return floor(t * gr.inv_q) * gr.q; }

// Host side: kernel launches that can carry timing events.  The library's
// timer may leave a (start, stop) pair here for the next launch made through
// launch() on this host thread; the pair then records that kernel's own start
// and end (hipExtLaunchKernel), without the gaps around the dispatch.
struct KernelEvents {
    hipEvent_t start, stop;
};
KernelEvents& pending_events();

template <typename F, typename... A>
inline void launch(F kernel, dim3 grid, dim3 block, size_t smem, hipStream_t st, A... args)
{
    KernelEvents& pe = pending_events();
    if (pe.start == nullptr) {
        kernel<<<grid, block, smem, st>>>(args...);
        return;
    }
    const KernelEvents ev = pe;
    pe = KernelEvents{nullptr, nullptr};
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)smem, st, ev.start, ev.stop, 0u, args...);
}

}  // namespace avl
