// Gather/push and the counting sort of markers by dual cell.
//
// One step's sort is three passes over the markers:
//   count   : (optionally) push each marker, find its new bucket, and count it;
//   scan    : exclusive prefix sum of the bucket counts -> run offsets;
//   scatter : push again (bit-identical arithmetic), claim a slot in the run,
//             and write the marker to its sorted position in the other buffer.
// Pushing twice instead of storing pushed positions between the passes saves
// a full write+read of the position/velocity streams; the push is a few
// flops per marker against 16-40 bytes of traffic.
//
// Counting uses integer atomics only.  A block's markers are contiguous in the
// previous sorted order, so after the push they land in a few neighbouring
// bucket rows; each block keeps a histogram of those rows in LDS and issues
// one global atomic per touched bucket.  Markers whose bucket falls outside
// that window (large velocity jumps) use one global atomic each.  The scatter
// uses the counts array itself as a descending cursor, which leaves it zeroed
// for the next step.
#include "avl_device.h"

namespace avl {

// ---------------------------------------------------------------------------
// Marker payloads and their bucket computation, per storage form.
// ---------------------------------------------------------------------------
template <int PREC, int VD> struct Pay;

template <int VD> struct Pay<0, VD> {
    double x, v[VD], f;
    __device__ void load(const M64& m, int n, int i, bool with_f) {
        x = m.x[i];
#pragma unroll
        for (int d = 0; d < VD; ++d) v[d] = m.v[(size_t)d * n + i];
        f = with_f ? m.f[i] : 0.0;
    }
    __device__ void store(const M64& m, int n, int i) const {
        m.x[i] = x;
#pragma unroll
        for (int d = 0; d < VD; ++d) m.v[(size_t)d * n + i] = v[d];
        m.f[i] = f;
    }
    __device__ void push(const Geo& g, const double* sE, const RowShift*, double dtk, float, int& flags) {
        push64(g, sE, dtk, x, v[0]);
        if (!isfinite(x) || !isfinite(v[0])) flags |= FLAG_NONFINITE;
    }
    __device__ int bucket(const Geo& g) const {
        int ix, jp[VD];
        double a, b[VD];
        return locate64<VD>(g, x, v, ix, jp, a, b);
    }
};

template <int VD> struct Pay<1, VD> {
    int cell;
    float a, b[VD], f;
    __device__ void load(const M32& m, int n, int i, bool with_f) {
        cell = m.cell[i];
        a = m.a[i];
#pragma unroll
        for (int d = 0; d < VD; ++d) b[d] = m.b[(size_t)d * n + i];
        f = with_f ? m.f[i] : 0.0f;
    }
    __device__ void store(const M32& m, int n, int i) const {
        m.cell[i] = cell;
        m.a[i] = a;
#pragma unroll
        for (int d = 0; d < VD; ++d) m.b[(size_t)d * n + i] = b[d];
        m.f[i] = f;
    }
    __device__ void push(const Geo& g, const float* sE, const RowShift* rows, double, float bk, int& flags) {
        push32<VD>(g, sE, rows, bk, cell, a, b[0], flags);
    }
    __device__ int bucket(const Geo& g) const { return bucket32<VD>(g, cell); }
};

template <int PREC> struct MarkersOf;
template <> struct MarkersOf<0> { using T = M64; using E = double; };
template <> struct MarkersOf<1> { using T = M32; using E = float; };

// The LDS window of a sort block: bucket rows around the rows of the block's
// first and last marker (which bound the block's rows, the input being
// sorted), widened by one row each way, at most hist_bins buckets.
__device__ __forceinline__ void set_window(const Geo& g, int b0, int b1, int* s_lo, int* s_nb)
{
    int r0 = (b0 >= g.nb ? g.nrow - 1 : b0 >> g.lognx);
    int r1 = (b1 >= g.nb ? g.nrow - 1 : b1 >> g.lognx);
    int lo = min(r0, r1) - 1, hi = max(r0, r1) + 1;
    lo = max(lo, 0);
    hi = min(hi, g.nrow - 1);
    int maxrows = g.hist_bins >> g.lognx;
    if (hi - lo + 1 > maxrows) hi = lo + maxrows - 1;
    *s_lo = lo << g.lognx;
    *s_nb = (hi - lo + 1) << g.lognx;
}

// Wavefront-aggregated LDS histogram update.  A wave holds 64 consecutive
// markers of the previous order, which land in only a handful of new buckets:
// lanes with equal bins are grouped with ballots, the first lane of each group
// adds the group size, and every lane gets its rank among all markers of its
// bin in this block (RANK) -- one conflict-free LDS atomic per distinct bin
// instead of one per marker.  `win` marks lanes with an in-window bin; all
// lanes of the wave must call this.
template <bool RANK>
__device__ __forceinline__ int wave_hist_add(int* hist, int rel, bool win)
{
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long pending = __ballot(win);
    int leader = 0, wrank = 0, cnt = 0;
    while (pending) {
        const int l = __ffsll((unsigned long long)pending) - 1;
        const int key = __shfl(rel, l, kWave);
        const unsigned long long same = __ballot(win && rel == key) & pending;
        if ((same >> lane) & 1ull) {
            leader = l;
            wrank = __popcll(same & below);
        }
        if (lane == l) cnt = __popcll(same);
        pending &= ~same;
    }
    int base = 0;
    if (cnt) {
        if (RANK) base = atomicAdd(&hist[rel], cnt);
        else atomicAdd(&hist[rel], cnt);
    }
    if (!RANK) return -1;
    base = __shfl(base, leader, kWave);
    return win ? base + wrank : -1;
}

template <int PREC>
__device__ void stage_field(const Geo& g, const double* E, typename MarkersOf<PREC>::E* sE)
{
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) sE[i] = (typename MarkersOf<PREC>::E)E[i];
}

template <int PREC>
struct SortSmem {
    typename MarkersOf<PREC>::E* sE;
    RowShift* sRow;
    int* hist;
    __device__ SortSmem(unsigned char* smem, const Geo& g) {
        using ET = typename MarkersOf<PREC>::E;
        sE = reinterpret_cast<ET*>(smem);
        sRow = reinterpret_cast<RowShift*>(smem + sizeof(ET) * g.nx);
        hist = reinterpret_cast<int*>(smem + sizeof(ET) * g.nx + (PREC ? sizeof(RowShift) * (g.nv[0] + 1) : 0));
    }
};

// Block prologue shared by count and scatter: stage the field (and drift
// table), find the histogram window from the already-loaded first and last
// markers, clear the window.  Marker loads are issued before this runs, so
// their latency overlaps the window set-up.
template <int PREC, int VD, int MPT, bool PUSH>
__device__ __forceinline__ void sort_prologue(const Geo& g, const SortSmem<PREC>& sm, const Pay<PREC, VD>* p,
                                              int base, int last, const double* E, const RowShift* rows_g,
                                              int* s_b, int* s_lo, int* s_nb)
{
    if (PUSH) {
        stage_field<PREC>(g, E, sm.sE);
        if (PREC)
            for (int i = threadIdx.x; i <= g.nv[0]; i += blockDim.x) sm.sRow[i] = rows_g[i];
    }
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        if (i == base) s_b[0] = p[k].bucket(g);
        if (i == last) s_b[1] = p[k].bucket(g);
    }
    __syncthreads();
    if (threadIdx.x == 0) set_window(g, s_b[0], s_b[1], s_lo, s_nb);
    __syncthreads();
    const int nbw = *s_nb;
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) sm.hist[i] = 0;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// count pass
// ---------------------------------------------------------------------------
template <int PREC, int VD, bool PUSH>
__global__ __launch_bounds__(kSortThreads) void k_count(Geo g, typename MarkersOf<PREC>::T m,
                                                        const double* __restrict__ E,
                                                        const RowShift* __restrict__ rows_g,
                                                        double dtk, float bk,
                                                        int* __restrict__ counts, int* __restrict__ flags)
{
    constexpr int MPT = kCountMPT;
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_lo, s_nb, s_flags;
    const int base = blockIdx.x * kCountTile;
    const int last = min(base + kCountTile, g.n) - 1;
    Pay<PREC, VD> p[MPT];
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        if (i <= last) p[k].load(m, g.n, i, false);
    }
    if (threadIdx.x == 0) s_flags = 0;
    sort_prologue<PREC, VD, MPT, PUSH>(g, sm, p, base, last, E, rows_g, s_b, &s_lo, &s_nb);
    const int lo = s_lo, nbw = s_nb;
    int fl = 0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        int rel = -1;
        bool win = false;
        if (i <= last) {
            if (PUSH) p[k].push(g, sm.sE, sm.sRow, dtk, bk, fl);
            const int bkt = p[k].bucket(g);
            rel = bkt - lo;
            win = rel >= 0 && rel < nbw;
            if (!win) atomicAdd(&counts[bkt], 1);
        }
        wave_hist_add<false>(sm.hist, rel, win);
    }
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) {
        const int c = sm.hist[i];
        if (c) atomicAdd(&counts[lo + i], c);
    }
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

// ---------------------------------------------------------------------------
// scatter pass: src (sorted by the previous buckets) -> dst (sorted by new)
// ---------------------------------------------------------------------------
template <int PREC, int VD, bool PUSH>
__global__ __launch_bounds__(kSortThreads) void k_scatter(Geo g, typename MarkersOf<PREC>::T src,
                                                          typename MarkersOf<PREC>::T dst,
                                                          const double* __restrict__ E,
                                                          const RowShift* __restrict__ rows_g,
                                                          double dtk, float bk,
                                                          const int* __restrict__ offsets,
                                                          int* __restrict__ counts, int* __restrict__ flags)
{
    constexpr int MPT = kSortMPT;
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_lo, s_nb, s_flags;
    const int base = blockIdx.x * kSortTile;
    const int last = min(base + kSortTile, g.n) - 1;
    Pay<PREC, VD> p[MPT];
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        if (i <= last) p[k].load(src, g.n, i, true);
    }
    if (threadIdx.x == 0) s_flags = 0;
    sort_prologue<PREC, VD, MPT, PUSH>(g, sm, p, base, last, E, rows_g, s_b, &s_lo, &s_nb);
    const int lo = s_lo, nbw = s_nb;
    int bkt[MPT], rank[MPT];
    int fl = 0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        bkt[k] = -1;
        int rel = -1;
        bool win = false;
        if (i <= last) {
            if (PUSH) p[k].push(g, sm.sE, sm.sRow, dtk, bk, fl);
            bkt[k] = p[k].bucket(g);
            rel = bkt[k] - lo;
            win = rel >= 0 && rel < nbw;
        }
        rank[k] = wave_hist_add<true>(sm.hist, rel, win);
    }
    __syncthreads();
    // claim each touched bucket's slots: counts[] holds the slots still free,
    // counting down from the run length
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) {
        const int c = sm.hist[i];
        if (c) {
            const int old = atomicSub(&counts[lo + i], c);
            int start = old - c;
            if (start < 0) { fl |= FLAG_SLOT; start = -1; }
            sm.hist[i] = start;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        if (bkt[k] < 0) continue;
        int slot;
        if (rank[k] >= 0) {
            const int start = sm.hist[bkt[k] - lo];
            slot = start < 0 ? -1 : start + rank[k];
        } else {
            slot = atomicSub(&counts[bkt[k]], 1) - 1;
        }
        const int beg = offsets[bkt[k]], end = offsets[bkt[k] + 1];
        const int dest = beg + slot;
        if (slot < 0 || dest >= end) { fl |= FLAG_SLOT; continue; }
        p[k].store(dst, g.n, dest);
    }
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

// ---------------------------------------------------------------------------
// order-preserving push (the standalone gather+push stage)
// ---------------------------------------------------------------------------
template <int PREC, int VD>
__global__ __launch_bounds__(kSortThreads) void k_push(Geo g, typename MarkersOf<PREC>::T m,
                                                       const double* __restrict__ E,
                                                       const RowShift* __restrict__ rows_g,
                                                       double dtk, float bk, int* __restrict__ flags)
{
    using ET = typename MarkersOf<PREC>::E;
    extern __shared__ __align__(16) unsigned char smem[];
    ET* sE = reinterpret_cast<ET*>(smem);
    RowShift* sRow = reinterpret_cast<RowShift*>(smem + sizeof(ET) * g.nx);
    stage_field<PREC>(g, E, sE);
    if (PREC)
        for (int i = threadIdx.x; i <= g.nv[0]; i += blockDim.x) sRow[i] = rows_g[i];
    __syncthreads();
    int fl = 0;
    const int base = blockIdx.x * kSortTile;
    for (int k = 0; k < kSortMPT; ++k) {
        int i = base + k * kSortThreads + threadIdx.x;
        if (i < g.n) {
            Pay<PREC, VD> p;
            p.load(m, g.n, i, true);
            p.push(g, sE, sRow, dtk, bk, fl);
            p.store(m, g.n, i);
        }
    }
    if (fl) atomicOr(flags, fl);
}

// ---------------------------------------------------------------------------
// exclusive scan of bucket counts (three phases over tiles of kScanTile)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ int block_excl_scan(int v, int* excl, int* s_w)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < nw; ++i) { int t = s_w[i]; s_w[i] = acc; acc += t; }
        s_w[nw] = acc;
    }
    __syncthreads();
    *excl = inc - v + s_w[w];
    int total = s_w[nw];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* __restrict__ counts, int nbt,
                                                             int* __restrict__ tile_sums)
{
    __shared__ int s_w[kScanThreads / kWave + 1];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        s += (i < nbt) ? counts[i] : 0;
    }
    int excl;
    int tot = block_excl_scan(s, &excl, s_w);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(int* __restrict__ tile_sums, int ntiles)
{
    __shared__ int s_w[1024 / kWave + 1];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < ntiles; base += blockDim.x) {
        int i = base + threadIdx.x;
        int v = i < ntiles ? tile_sums[i] : 0;
        int excl;
        int tot = block_excl_scan(v, &excl, s_w);
        if (i < ntiles) tile_sums[i] = excl + s_carry;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int* __restrict__ counts, int nbt,
                                                            const int* __restrict__ tile_excl,
                                                            int* __restrict__ offsets)
{
    __shared__ int s_w[kScanThreads / kWave + 1];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int c[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        c[k] = (i < nbt) ? counts[i] : 0;
        s += c[k];
    }
    int excl;
    block_excl_scan(s, &excl, s_w);
    int run = excl + tile_excl[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int i = base + k;
        if (i < nbt) offsets[i] = run;
        run += c[k];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int PREC>
static size_t sort_smem(const Geo& g, bool push)
{
    size_t e = push ? (PREC ? sizeof(float) : sizeof(double)) * g.nx : (PREC ? sizeof(float) : sizeof(double)) * g.nx;
    size_t r = PREC ? sizeof(RowShift) * (g.nv[0] + 1) : 0;
    return e + r + sizeof(int) * g.hist_bins;
}

template <int PREC, int VD>
static hipError_t launch_sort_t(const Geo& g, void* src, void* dst, const double* E, const RowShift* rows,
                                double dtk, float bk, int* counts, int* offsets, int* tile_sums,
                                int* flags, bool push, hipStream_t st, int phase)
{
    using MT = typename MarkersOf<PREC>::T;
    MT s = *reinterpret_cast<MT*>(src);
    MT d = dst ? *reinterpret_cast<MT*>(dst) : s;
    const int cblocks = (g.n + kCountTile - 1) / kCountTile;
    const int sblocks = (g.n + kSortTile - 1) / kSortTile;
    const size_t smem = sort_smem<PREC>(g, push);
    if (g.n == 0 && phase != 1) return hipSuccess;   // the scan still runs: offsets become zero
    static int granted[4] = {0, 0, 0, 0};
    {
        const void* fns[4] = {(const void*)k_count<PREC, VD, true>, (const void*)k_count<PREC, VD, false>,
                              (const void*)k_scatter<PREC, VD, true>, (const void*)k_scatter<PREC, VD, false>};
        for (int i = 0; i < 4; ++i) {
            hipError_t e = ensure_lds(fns[i], smem, granted[i]);
            if (e != hipSuccess) return e;
        }
    }
    if (phase == 0) {
        if (push) hipLaunchKernelGGL((k_count<PREC, VD, true>), dim3(cblocks), dim3(kSortThreads), smem, st, g, s, E, rows, dtk, bk, counts, flags);
        else hipLaunchKernelGGL((k_count<PREC, VD, false>), dim3(cblocks), dim3(kSortThreads), smem, st, g, s, E, rows, dtk, bk, counts, flags);
    } else if (phase == 1) {
        const int nbt = g.nb + 1;
        const int ntiles = (nbt + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_reduce, dim3(ntiles), dim3(kScanThreads), 0, st, counts, nbt, tile_sums);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tile_sums, ntiles);
        hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, st, counts, nbt, tile_sums, offsets);
    } else {
        if (push) hipLaunchKernelGGL((k_scatter<PREC, VD, true>), dim3(sblocks), dim3(kSortThreads), smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags);
        else hipLaunchKernelGGL((k_scatter<PREC, VD, false>), dim3(sblocks), dim3(kSortThreads), smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags);
    }
    return hipGetLastError();
}

// phase 0 = count, 1 = scan, 2 = scatter
hipError_t launch_sort(const Geo& g, void* src, void* dst, const double* E, const RowShift* rows,
                       double dtk, float bk, int* counts, int* offsets, int* tile_sums, int* flags,
                       bool push, hipStream_t st, int phase)
{
    if (g.prec == 0 && g.vdim == 1) return launch_sort_t<0, 1>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, flags, push, st, phase);
    if (g.prec == 0 && g.vdim == 3) return launch_sort_t<0, 3>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, flags, push, st, phase);
    if (g.prec == 1 && g.vdim == 1) return launch_sort_t<1, 1>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, flags, push, st, phase);
    return launch_sort_t<1, 3>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, flags, push, st, phase);
}

hipError_t launch_push(const Geo& g, void* m, const double* E, const RowShift* rows, double dtk, float bk,
                       int* flags, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const int blocks = (g.n + kSortTile - 1) / kSortTile;
    const size_t smem = (g.prec ? sizeof(float) : sizeof(double)) * g.nx + (g.prec ? sizeof(RowShift) * (g.nv[0] + 1) : 0);
    if (g.prec == 0 && g.vdim == 1) hipLaunchKernelGGL((k_push<0, 1>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M64*>(m), E, rows, dtk, bk, flags);
    else if (g.prec == 0) hipLaunchKernelGGL((k_push<0, 3>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M64*>(m), E, rows, dtk, bk, flags);
    else if (g.vdim == 1) hipLaunchKernelGGL((k_push<1, 1>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M32*>(m), E, rows, dtk, bk, flags);
    else hipLaunchKernelGGL((k_push<1, 3>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M32*>(m), E, rows, dtk, bk, flags);
    return hipGetLastError();
}

}  // namespace avl
