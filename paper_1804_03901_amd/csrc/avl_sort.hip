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
//
// Implied cells (FP32 1D-1V).  In that form a marker's cell index equals its
// bucket whenever its cloud touches the grid, and once sorted, a marker's
// bucket is the run its position falls in.  So the scatter stores the cell
// index only for markers of the overflow bucket, and the next sort recovers
// every other cell from the previous run offsets: per tile, the starts of the
// runs inside it are marked in LDS and a block-wide running maximum fills in
// the rest (the scan also records the bucket of every kTfStride-th position,
// where each tile starts).  That is 4 bytes a marker less to read in the count
// and the scatter and to write in the scatter.
#include <algorithm>

#include "avl_device.h"

namespace avl {

// ---------------------------------------------------------------------------
// Marker payloads and their bucket computation, per storage form.  Component
// arrays are laid out with the padded stride g.np (a multiple of 64 markers),
// so a thread's group of consecutive markers can be read with 16-byte loads.
// ---------------------------------------------------------------------------
template <int PREC, int VD> struct Pay;

template <int VD> struct Pay<0, VD> {
    double x, v[VD], f;
    int id;
    __device__ void load(const M64& m, const Geo& g, int i, bool with_f, int = VD, bool = true) {
        x = m.x[i];
#pragma unroll
        for (int d = 0; d < VD; ++d) v[d] = m.v[(size_t)d * g.np + i];
        f = with_f ? m.f[i] : 0.0;
        id = (with_f && m.id) ? m.id[i] : 0;
    }
    __device__ void store(const M64& m, const Geo& g, int i, bool = true) const {
        m.x[i] = x;
#pragma unroll
        for (int d = 0; d < VD; ++d) m.v[(size_t)d * g.np + i] = v[d];
        m.f[i] = f;
        if (m.id) m.id[i] = id;
    }
    __device__ void push(const Geo& g, const double* sE, const RowShift*, double dtk, float, int& flags) {
        push64<VD>(g, sE, dtk, x, v);
        bool ok = isfinite(x) && isfinite(v[0]);
        if (VD == 3 && g.magnetic) ok = ok && isfinite(v[1]) && isfinite(v[2]);
        if (!ok) flags |= FLAG_NONFINITE;
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
    int id;
    // nvel < VD loads only the first nvel velocity offsets; with_cell false
    // leaves the cell index to be filled in from the previous run offsets
    __device__ void load(const M32& m, const Geo& g, int i, bool with_f, int nvel = VD, bool with_cell = true) {
        cell = with_cell ? m.cell[i] : 0;
        a = m.a[i];
#pragma unroll
        for (int d = 0; d < VD; ++d) b[d] = d < nvel ? m.b[(size_t)d * g.np + i] : 0.0f;
        f = with_f ? m.f[i] : 0.0f;
        id = (with_f && m.id) ? m.id[i] : 0;
    }
    // all_cells false (the sort's output in 1D-1V): the cell index is written
    // only for markers of the overflow bucket, the others being implied by
    // the run offsets of the new order
    __device__ void store(const M32& m, const Geo& g, int i, bool all_cells = true) const {
        if (all_cells || VD != 1 || bucket32<VD>(g, cell) == g.nb) m.cell[i] = cell;
        m.a[i] = a;
#pragma unroll
        for (int d = 0; d < VD; ++d) m.b[(size_t)d * g.np + i] = b[d];
        m.f[i] = f;
        if (m.id) m.id[i] = id;
    }
    __device__ void push(const Geo& g, const float2* sE, const RowShift* rows, double, float, int& flags) {
        push32<VD>(g, sE, rows, cell, a, b[0], flags);
    }
    __device__ int bucket(const Geo& g) const { return bucket32<VD>(g, cell); }
};

template <int PREC> struct MarkersOf;
template <> struct MarkersOf<0> { using T = M64; using E = double; };
template <> struct MarkersOf<1> { using T = M32; using E = float2; };   // E: staged field (kick, difference)

// K consecutive elements starting at a 16-byte aligned address, as 16-byte loads.
template <typename T, int K>
__device__ __forceinline__ void vload(const T* __restrict__ src, T* out)
{
    static_assert((K * sizeof(T)) % 16 == 0, "group must be a multiple of 16 bytes");
    constexpr int V = 16 / sizeof(T);
#pragma unroll
    for (int j = 0; j < K / V; ++j) {
        const int4 t = *reinterpret_cast<const int4*>(src + j * V);
        __builtin_memcpy(out + j * V, &t, 16);
    }
}

// A thread's group of K consecutive markers [first, first+K), all loads issued
// together.  Past the last marker, indices are clamped (values masked later).
template <int PREC, int VD, int K> struct Group;

template <int VD, int K> struct Group<0, VD, K> {
    Pay<0, VD> p[K];
    __device__ void load(const M64& m, const Geo& g, int first, int last, bool with_f, int = VD, int = -1) {
        if (first + K - 1 <= last) {
            double t[K];
            vload<double, K>(m.x + first, t);
#pragma unroll
            for (int k = 0; k < K; ++k) p[k].x = t[k];
#pragma unroll
            for (int d = 0; d < VD; ++d) {
                vload<double, K>(m.v + (size_t)d * g.np + first, t);
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].v[d] = t[k];
            }
            if (with_f) {
                vload<double, K>(m.f + first, t);
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].f = t[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) p[k].load(m, g, min(first + k, last), with_f);
        }
    }
};

template <int VD, int K> struct Group<1, VD, K> {
    Pay<1, VD> p[K];
    // nvel < VD loads only the first nvel velocity offsets (the count pass
    // needs the cell index, a and the x-velocity offset only).  ovf >= 0:
    // implied cells, read from memory only at positions >= ovf (the
    // overflow run of the previous order); the rest are filled in later.
    __device__ void load(const M32& m, const Geo& g, int first, int last, bool with_f, int nvel = VD, int ovf = -1) {
        if (first + K - 1 <= last) {
            int ti[K];
            float t[K];
            if (ovf < 0) {
                vload<int, K>(m.cell + first, ti);
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].cell = ti[k];
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].cell = 0;
                if (first + K - 1 >= ovf) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (first + k >= ovf) p[k].cell = m.cell[first + k];
                }
            }
            vload<float, K>(m.a + first, t);
#pragma unroll
            for (int k = 0; k < K; ++k) p[k].a = t[k];
#pragma unroll
            for (int d = 0; d < VD; ++d) {
                if (d < nvel) {
                    vload<float, K>(m.b + (size_t)d * g.np + first, t);
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) t[k] = 0.0f;
                }
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].b[d] = t[k];
            }
            if (with_f) {
                vload<float, K>(m.f + first, t);
#pragma unroll
                for (int k = 0; k < K; ++k) p[k].f = t[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = min(first + k, last);
                p[k].load(m, g, i, with_f, nvel, ovf < 0 || i >= ovf);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Implied cells: the previous order's buckets of one tile's positions.
// ---------------------------------------------------------------------------
constexpr int kTfLog = 11;                   // the scan records the bucket of every 2^kTfLog-th position
constexpr int kTfStride = 1 << kTfLog;
static_assert(kSortTile == kTfStride && kCountTile % kTfStride == 0, "tiles start at recorded positions");

// The order the markers are in, for implied cells: its run offsets (nb + 2
// entries) and the bucket of every kTfStride-th position.  off == nullptr:
// the cell indices are all stored.
struct Prev {
    const int* off;
    const int* tfirst;
};

// Run offsets of tile_buckets' first pass, loaded ahead of the tile: b0, the
// run that holds the tile's first position, and the bounds of run b0 + 1 + t
// for thread t (zero past the last run).
struct TbAhead {
    int b0, lo, hi;
};

__device__ __forceinline__ int tile_first_run(const Prev& pv, int base) { return pv.tfirst[base >> kTfLog]; }

__device__ __forceinline__ TbAhead tile_runs_ahead(const Geo& g, const Prev& pv, int b0)
{
    TbAhead a{b0, 0, 0};
    // clamped: tiles past the start of the overflow run load this too
    const int b = min(max(b0, 0), g.nb) + 1 + (int)threadIdx.x;
    if (b < g.nb) {
        a.lo = pv.off[b];
        a.hi = pv.off[b + 1];
    }
    return a;
}

// Buckets of the positions [base, end) of a tile (base a multiple of
// kTfStride, end at most the start of the overflow run): the largest b with
// off[b] <= p.  Thread t owns the SL slots [t SL, t SL + SL) of `map` (T =
// kSortThreads SL ints of LDS, free on entry) and gets their buckets in bk[]
// (undefined past end); with WRITE they are also left in map for other
// threads, after a barrier.  s_aux: kSortThreads / kWave + 1 ints of LDS.
// AHEAD: the first pass takes b0 and its offsets from ah instead of loading them.
template <int SL, bool WRITE, bool AHEAD = false>
__device__ __forceinline__ void tile_buckets(const Geo& g, const Prev& pv, int base, int end, int* map, int* s_aux,
                                             int (&bk)[SL], const TbAhead& ah = TbAhead{0, 0, 0})
{
    static_assert(SL % 4 == 0, "slots are cleared and read as 16-byte vectors");
    const int tid = threadIdx.x;
    const int b0 = AHEAD ? ah.b0 : tile_first_run(pv, base);   // the run that holds position base
    // the LDS is the previous tile's histogram, which its last stores may
    // still be reading (a block walks several tiles)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SL; k += 4) *reinterpret_cast<int4*>(map + tid * SL + k) = make_int4(-1, -1, -1, -1);
    if (tid == 0) map[0] = b0;
    __syncthreads();
    // mark the start of every later run that begins inside the tile
    for (int bs = b0 + 1;; bs += kSortThreads) {
        const int b = bs + tid;
        int lo = end;
        if (b < g.nb) {
            int hi;
            if (AHEAD && bs == b0 + 1) {
                lo = ah.lo;
                hi = ah.hi;
            } else {
                lo = pv.off[b];
                hi = pv.off[b + 1];
            }
            if (lo < hi && lo > base && lo < end) map[lo - base] = b;
        }
        if (tid == kSortThreads - 1) s_aux[kSortThreads / kWave] = (b < g.nb && lo < end) ? 1 : 0;
        __syncthreads();
        const int more = s_aux[kSortThreads / kWave];
        if (!more) break;
        // the flag is written again by the next pass
        __syncthreads();
    }
    // running maximum over the slots: within the thread, then across threads
#pragma unroll
    for (int k = 0; k < SL; k += 4) {
        const int4 v = *reinterpret_cast<const int4*>(map + tid * SL + k);
        bk[k] = v.x; bk[k + 1] = v.y; bk[k + 2] = v.z; bk[k + 3] = v.w;
    }
#pragma unroll
    for (int k = 1; k < SL; ++k) bk[k] = max(bk[k], bk[k - 1]);
    const int lane = tid & (kWave - 1), w = tid / kWave;
    int inc = bk[SL - 1];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc = max(inc, t);
    }
    int carry = __shfl_up(inc, 1, kWave);
    if (lane == 0) carry = -1;
    if (lane == kWave - 1) s_aux[w] = inc;
    __syncthreads();
    for (int q = 0; q < w; ++q) carry = max(carry, s_aux[q]);
#pragma unroll
    for (int k = 0; k < SL; ++k) bk[k] = max(bk[k], carry);
    if constexpr (WRITE) {
#pragma unroll
        for (int k = 0; k < SL; k += 4)
            *reinterpret_cast<int4*>(map + tid * SL + k) = make_int4(bk[k], bk[k + 1], bk[k + 2], bk[k + 3]);
        __syncthreads();
    }
}

// The LDS window of a sort block: bucket rows around the rows of the block's
// first and last marker (which bound the block's rows, the input being
// sorted), widened by one row each way, at most maxbins buckets.
__device__ __forceinline__ void set_window(const Geo& g, int b0, int b1, int* lo_out, int* nb_out, int maxbins)
{
    int r0 = (b0 >= g.nb ? g.nrow - 1 : b0 >> g.lognx);
    int r1 = (b1 >= g.nb ? g.nrow - 1 : b1 >> g.lognx);
    int lo = min(r0, r1) - 1, hi = max(r0, r1) + 1;
    lo = max(lo, 0);
    hi = min(hi, g.nrow - 1);
    int maxrows = maxbins >> g.lognx;
    if (hi - lo + 1 > maxrows) hi = lo + maxrows - 1;
    *lo_out = lo << g.lognx;
    *nb_out = (hi - lo + 1) << g.lognx;
}

// Stage the field and, in the FP32 form, the drift table into LDS.  The FP64
// path stages E itself; the FP32 form stages the kick in units of dv,
// e_i = E_i * bk rounded once from FP64, with its forward difference
// e_{i+1} - e_i.  Each thread issues all its loads before its first LDS
// store, so staging costs one round trip to L2 instead of one per element.
template <int PREC>
__device__ __forceinline__ void stage_tables(const Geo& g, typename MarkersOf<PREC>::E* sE, RowShift* sRow,
                                             const double* __restrict__ E, const RowShift* __restrict__ rows_g,
                                             float bk)
{
    constexpr int U = 8;
    const int nr = PREC ? g.nv[0] + 1 : 0;
    const int span = U * (int)blockDim.x;
    const int ntot = max(g.nx, nr);
    for (int i0 = 0; i0 < ntot; i0 += span) {
        double e[U], e1[U];
        RowShift r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
            e[u] = i < g.nx ? E[i] : 0.0;
            if (PREC) {
                e1[u] = i < g.nx ? E[(i + 1) & (g.nx - 1)] : 0.0;
                r[u] = i < nr ? rows_g[i] : RowShift{0, 0.0f};
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
            if constexpr (PREC) {
                const float k0 = (float)(e[u] * (double)bk), k1 = (float)(e1[u] * (double)bk);
                if (i < g.nx) sE[i] = make_float2(k0, k1 - k0);
                if (i < nr) sRow[i] = r[u];
            } else {
                if (i < g.nx) sE[i] = e[u];
            }
        }
    }
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
        // 16-byte aligned: the implied-cell map is accessed as int4
        const size_t h = (sizeof(ET) * g.nx + (PREC ? sizeof(RowShift) * (g.nv[0] + 1) : 0) + 15) & ~(size_t)15;
        hist = reinterpret_cast<int*>(smem + h);
    }
};

// Per-thread aggregation of a group's buckets.  Consecutive markers of the
// previous order come from one or two runs and land in a few new buckets, so a
// thread keeps two "open" buckets with counts and gives each marker its rank
// inside its open bucket (tag 0 or 1); any further bucket is an "extra"
// (tag 2) handled one marker at a time.
template <int K>
struct Agg {
    int b0, b1, c0, c1;
    int tag[K], r[K];
    __device__ void build(const int* bkt) {
        b0 = -1; b1 = -1; c0 = 0; c1 = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int b = bkt[k];
            tag[k] = -1;
            r[k] = 0;
            if (b < 0) continue;
            if (b0 < 0 || b == b0) { b0 = b; tag[k] = 0; r[k] = c0++; }
            else if (b1 < 0 || b == b1) { b1 = b; tag[k] = 1; r[k] = c1++; }
            else tag[k] = 2;
        }
    }
};

// ---------------------------------------------------------------------------
// count pass
// ---------------------------------------------------------------------------
// One tile of the count pass: the thread's group of K consecutive markers
// [first, first+K) of the tile [base, last] is in grp (previous order), the
// field and drift table staged in LDS.
template <int PREC, int VD, bool PUSH, bool IMPL, bool AHEAD = false>
__device__ __forceinline__ void count_tile(const Geo& g, const SortSmem<PREC>& sm, Group<PREC, VD, count_mpt<PREC>()>& grp,
                                           double dtk, float bk, int* __restrict__ counts, int* __restrict__ tsum,
                                           int base, int last, int* s_b, int* s_tile, int& fl,
                                           const Prev& pv, int ovf, int* s_aux, const TbAhead& ah = TbAhead{0, 0, 0})
{
    constexpr int K = count_mpt<PREC>();
    const int first = base + threadIdx.x * K;
    if constexpr (IMPL) {
        // implied cells: this thread's K consecutive positions are its own slots
        int ob[K];
        if (base < ovf) {
            tile_buckets<K, false, AHEAD>(g, pv, base, min(last + 1, ovf), sm.hist, s_aux, ob, ah);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (first + k < ovf) grp.p[k].cell = ob[k];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (first + k == base) s_b[0] = grp.p[k].bucket(g);
        if (first + k == last) s_b[1] = grp.p[k].bucket(g);
    }
    __syncthreads();
    // every thread forms the window from the tile's two end buckets itself
    int lo, nbw;
    set_window(g, s_b[0], s_b[1], &lo, &nbw, g.hist_bins);
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) sm.hist[i] = 0;
    if (threadIdx.x < 8) s_tile[threadIdx.x] = 0;
    __syncthreads();
    int bkt[K];
    if constexpr (PUSH && PREC == 1 && VD == 1) {
        // 1D-1V FP32 form: only the new buckets; past the last marker the
        // group holds copies of it, pushed too (the markers' LDS round trips
        // interleave) and not counted.  The flags are raised by the scatter,
        // which pushes the same markers with the same field.
        int c[K];
        float a[K], b[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            c[k] = grp.p[k].cell;
            a[k] = grp.p[k].a;
            b[k] = grp.p[k].b[0];
        }
        push32_buckets<K>(g, sm.sE, sm.sRow, c, a, b, bkt);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (first + k > last) bkt[k] = -1;
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // FP32 form: as above, copies of the last marker are pushed too
            if (PUSH && (PREC == 1 || first + k <= last)) grp.p[k].push(g, sm.sE, sm.sRow, dtk, bk, fl);
            bkt[k] = first + k <= last ? grp.p[k].bucket(g) : -1;
        }
    }
    Agg<K> ag;
    ag.build(bkt);
    auto add = [&](int b, int c) {
        const int rel = b - lo;
        if (rel >= 0 && rel < nbw) {
            atomicAdd(&sm.hist[rel], c);
        } else {
            atomicAdd(&counts[b], c);
            atomicAdd(&tsum[b / kScanTile], c);
        }
    };
    if (ag.c0) add(ag.b0, ag.c0);
    if (ag.c1) add(ag.b1, ag.c1);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (ag.tag[k] == 2) add(bkt[k], 1);
    __syncthreads();
    // flush the window; the same counts also go into per-scan-tile totals
    // (kScanTile buckets each), so the scan needs no separate reduction pass
    const int tlo = lo / kScanTile;
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) {
        const int c = sm.hist[i];
        if (c) {
            atomicAdd(&counts[lo + i], c);
            atomicAdd(&s_tile[(lo + i) / kScanTile - tlo], c);
        }
    }
    __syncthreads();
    const int ntile_win = (lo + nbw - 1) / kScanTile - tlo + 1;
    if (threadIdx.x < ntile_win && s_tile[threadIdx.x]) atomicAdd(&tsum[tlo + threadIdx.x], s_tile[threadIdx.x]);
}

// Tile t of the count pass covers markers [t*T, ...), T = count_tile_size; in
// the FP32 form the push needs the velocity offset b[0] only.
template <int PREC>
__device__ __forceinline__ int count_tile_last(const Geo& g, int t)
{
    constexpr int T = kSortThreads * count_mpt<PREC>();
    return min(t * T + T, g.n) - 1;
}

// count pass of one block over one tile (the batched kernel and the forms
// without a tiled kernel)
template <int PREC, int VD, bool PUSH, bool IMPL>
__device__ __forceinline__ void count_block(const Geo& g, const typename MarkersOf<PREC>::T& m,
                                            const double* __restrict__ E, const RowShift* __restrict__ rows_g,
                                            double dtk, float bk, int* __restrict__ counts, int* __restrict__ tsum,
                                            int* __restrict__ flags, int blk, const Prev& pv)
{
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_flags, s_tile[8], s_aux[kSortThreads / kWave + 1];
    if (threadIdx.x == 0) s_flags = 0;
    if (PUSH) stage_tables<PREC>(g, sm.sE, sm.sRow, E, rows_g, bk);
    constexpr int K = count_mpt<PREC>();
    Group<PREC, VD, K> grp;
    const int base = blk * (kSortThreads * K);
    const int last = count_tile_last<PREC>(g, blk);
    const int ovf = IMPL ? pv.off[g.nb] : -1;
    grp.load(m, g, base + threadIdx.x * K, last, false, PREC ? 1 : VD, ovf);
    int fl = 0;
    count_tile<PREC, VD, PUSH, IMPL>(g, sm, grp, dtk, bk, counts, tsum, base, last, s_b, s_tile, fl, pv,
                                     ovf, s_aux);
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

template <int PREC, int VD, bool PUSH>
__global__ __launch_bounds__(kSortThreads) void k_count(Geo g, typename MarkersOf<PREC>::T m,
                                                         const double* __restrict__ E,
                                                         const RowShift* __restrict__ rows_g,
                                                         double dtk, float bk,
                                                         int* __restrict__ counts, int* __restrict__ tsum,
                                                         int* __restrict__ flags)
{
    count_block<PREC, VD, PUSH, false>(g, m, E, rows_g, dtk, bk, counts, tsum, flags, blockIdx.x, Prev{nullptr, nullptr});
}

// Tiled count pass: each block takes tiles blockIdx.x, blockIdx.x + gridDim.x,
// ... (one block per resident slot), so the field and drift table are staged
// once per block instead of once per tile.
template <int PREC, int VD, bool PUSH, bool IMPL>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_count_tiled(Geo g, typename MarkersOf<PREC>::T m,
                                                         const double* __restrict__ E,
                                                         const RowShift* __restrict__ rows_g,
                                                         double dtk, float bk,
                                                         int* __restrict__ counts, int* __restrict__ tsum,
                                                         int* __restrict__ flags, Prev pv)
{
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_flags, s_tile[8], s_aux[kSortThreads / kWave + 1];
    constexpr int K = count_mpt<PREC>();
    constexpr int T = kSortThreads * K;
    const int ntiles = (g.n + T - 1) / T;
    const int ovf = IMPL ? pv.off[g.nb] : -1;
    if (threadIdx.x == 0) s_flags = 0;
    if (PUSH) stage_tables<PREC>(g, sm.sE, sm.sRow, E, rows_g, bk);
    int fl = 0;
    // implied cells: a tile's first-pass run offsets are loaded one tile
    // ahead, its first run two tiles ahead (as in the scatter)
    TbAhead ah{0, 0, 0};
    int b0n = 0;
    if constexpr (IMPL) {
        if ((int)blockIdx.x < ntiles) ah = tile_runs_ahead(g, pv, tile_first_run(pv, blockIdx.x * T));
        if ((int)(blockIdx.x + gridDim.x) < ntiles) b0n = tile_first_run(pv, (blockIdx.x + gridDim.x) * T);
    }
    const int my_tiles = (ntiles - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        prio_by_progress((t - (int)blockIdx.x) / (int)gridDim.x, my_tiles);
        Group<PREC, VD, K> grp;
        const int last = count_tile_last<PREC>(g, t);
        grp.load(m, g, t * T + threadIdx.x * K, last, false, PREC ? 1 : VD, ovf);
        TbAhead an{0, 0, 0};
        if constexpr (IMPL) {
            const int tn = t + gridDim.x, tnn = tn + gridDim.x;
            if (tn < ntiles) an = tile_runs_ahead(g, pv, b0n);
            if (tnn < ntiles) b0n = tile_first_run(pv, tnn * T);
        }
        count_tile<PREC, VD, PUSH, IMPL, IMPL>(g, sm, grp, dtk, bk, counts, tsum, t * T, last, s_b,
                                               s_tile, fl, pv, ovf, s_aux, ah);
        ah = an;
    }
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

// ---------------------------------------------------------------------------
// scatter pass: src (sorted by the previous buckets) -> dst (sorted by new)
//
// Here consecutive lanes take consecutive markers (lane-strided), unlike the
// count pass: markers of one previous run sit in neighbouring lanes and get
// consecutive ranks in their new run from the LDS atomics, so each store
// instruction writes a few contiguous stretches instead of 64 scattered words.
// ---------------------------------------------------------------------------
// One tile of the scatter: the markers [base, last] of the previous order are
// in p[] (lane-strided), the field and drift table staged in LDS.
template <int PREC, int VD, bool PUSH, bool IMPL, bool AHEAD = false>
__device__ __forceinline__ void scatter_tile(const Geo& g, const SortSmem<PREC>& sm, Pay<PREC, VD>* p,
                                             const typename MarkersOf<PREC>::T& dst, double dtk, float bk,
                                             const int* __restrict__ offsets, int* __restrict__ counts,
                                             int base, int last, int* s_b, int& fl,
                                             const Prev& pv, int ovf, int* s_aux, int maxbins,
                                             const TbAhead& ah = TbAhead{0, 0, 0})
{
    constexpr int K = kSortMPT;
    if constexpr (IMPL) {
        // implied cells: the tile's buckets are left in LDS, read lane-strided
        if (base < ovf) {
            int ob[K];
            tile_buckets<K, true, AHEAD>(g, pv, base, min(last + 1, ovf), sm.hist, s_aux, ob, ah);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int i = base + k * kSortThreads + threadIdx.x;
                if (i <= last && i < ovf) p[k].cell = sm.hist[i - base];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        if (i == base) s_b[0] = p[k].bucket(g);
        if (i == last) s_b[1] = p[k].bucket(g);
    }
    __syncthreads();
    // every thread forms the window from the tile's two end buckets itself
    int lo, nbw;
    set_window(g, s_b[0], s_b[1], &lo, &nbw, maxbins);
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) sm.hist[i] = 0;
    __syncthreads();
    int bkt[K], rank[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = base + k * kSortThreads + threadIdx.x;
        bkt[k] = -1;
        rank[k] = -1;
        if (i <= last) {
            if (PUSH) p[k].push(g, sm.sE, sm.sRow, dtk, bk, fl);
            bkt[k] = p[k].bucket(g);
            const int rel = bkt[k] - lo;
            if (rel >= 0 && rel < nbw) rank[k] = atomicAdd(&sm.hist[rel], 1);
        }
    }
    __syncthreads();
    // claim each touched in-window bucket's slots: counts[] holds the slots
    // still free, counting down from the run length, so a claim that starts
    // at or above zero lies inside the run; the histogram entry becomes the
    // first claimed position
    for (int i = threadIdx.x; i < nbw; i += blockDim.x) {
        const int c = sm.hist[i];
        if (c) {
            const int old = atomicSub(&counts[lo + i], c);
            const int start = old - c;
            if (start < 0) fl |= FLAG_SLOT;
            sm.hist[i] = start < 0 ? -1 : offsets[lo + i] + start;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (bkt[k] < 0) continue;
        int dest;
        if (rank[k] >= 0) {
            const int first = sm.hist[bkt[k] - lo];
            dest = first < 0 ? -1 : first + rank[k];
        } else {
            // outside the window (a large velocity jump): one slot at a time
            const int slot = atomicSub(&counts[bkt[k]], 1) - 1;
            dest = slot < 0 ? -1 : offsets[bkt[k]] + slot;
        }
        if (dest < 0) { fl |= FLAG_SLOT; continue; }
        p[k].store(dst, g, dest, false);
    }
}

// ovf >= 0: implied cells, stored only at positions >= ovf
template <int PREC, int VD>
__device__ __forceinline__ void load_tile(const typename MarkersOf<PREC>::T& src, const Geo& g, Pay<PREC, VD>* p,
                                          int base, int last, int ovf = -1, bool with_f = true)
{
#pragma unroll
    for (int k = 0; k < kSortMPT; ++k) {
        const int i = min(base + k * kSortThreads + (int)threadIdx.x, last);
        p[k].load(src, g, i, with_f, VD, ovf < 0 || i >= ovf);
    }
}

// scatter pass of one block over one tile (the batched kernel and the forms
// without a tiled kernel)
template <int PREC, int VD, bool PUSH, bool IMPL>
__device__ __forceinline__ void scatter_block(const Geo& g, const typename MarkersOf<PREC>::T& src,
                                              const typename MarkersOf<PREC>::T& dst,
                                              const double* __restrict__ E, const RowShift* __restrict__ rows_g,
                                              double dtk, float bk, const int* __restrict__ offsets,
                                              int* __restrict__ counts, int* __restrict__ flags, int blk, const Prev& pv,
                                              int maxbins)
{
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_flags, s_aux[kSortThreads / kWave + 1];
    const int base = blk * kSortTile;
    const int last = min(base + kSortTile, g.n) - 1;
    const int ovf = IMPL ? pv.off[g.nb] : -1;
    if (threadIdx.x == 0) s_flags = 0;
    if (PUSH) stage_tables<PREC>(g, sm.sE, sm.sRow, E, rows_g, bk);
    Pay<PREC, VD> p[kSortMPT];
    load_tile<PREC, VD>(src, g, p, base, last, ovf);
    int fl = 0;
    scatter_tile<PREC, VD, PUSH, IMPL>(g, sm, p, dst, dtk, bk, offsets, counts, base, last, s_b, fl,
                                       pv, ovf, s_aux, maxbins);
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

template <int PREC, int VD, bool PUSH>
__global__ __launch_bounds__(kSortThreads) void k_scatter1(Geo g, typename MarkersOf<PREC>::T src,
                                                           typename MarkersOf<PREC>::T dst,
                                                           const double* __restrict__ E,
                                                           const RowShift* __restrict__ rows_g,
                                                           double dtk, float bk,
                                                           const int* __restrict__ offsets,
                                                           int* __restrict__ counts, int* __restrict__ flags)
{
    scatter_block<PREC, VD, PUSH, false>(g, src, dst, E, rows_g, dtk, bk, offsets, counts, flags, blockIdx.x,
                                         Prev{nullptr, nullptr}, g.hist_bins);
}

// Tiled scatter: each block takes tiles blockIdx.x, blockIdx.x + gridDim.x,
// ... and loads its next tile's markers while the current one is pushed,
// ranked, claimed and stored, so the loads of one tile overlap the latency
// chain of the previous one; the field and drift table are staged once.
// ID false: the markers carry no identities (every run but an adjoint's), so
// the payload holds no id register (the null pointers are known at compile
// time).
template <int PREC, int VD, bool PUSH, bool IMPL, bool ID>
__device__ __forceinline__ void scatter_tiled(const Geo& g, typename MarkersOf<PREC>::T src,
                                              typename MarkersOf<PREC>::T dst, const double* __restrict__ E,
                                              const RowShift* __restrict__ rows_g, double dtk, float bk,
                                              const int* __restrict__ offsets, int* __restrict__ counts,
                                              int* __restrict__ flags, const Prev& pv)
{
    if constexpr (!ID) {
        src.id = nullptr;
        dst.id = nullptr;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    SortSmem<PREC> sm(smem, g);
    __shared__ int s_b[2], s_flags, s_aux[kSortThreads / kWave + 1];
    const int ntiles = (g.n + kSortTile - 1) / kSortTile;
    const int ovf = IMPL ? pv.off[g.nb] : -1;
    if (threadIdx.x == 0) s_flags = 0;
    if (PUSH) stage_tables<PREC>(g, sm.sE, sm.sRow, E, rows_g, bk);
    int fl = 0;
    Pay<PREC, VD> p[kSortMPT], q[kSortMPT];
    int t = blockIdx.x;
    // f is only needed when the marker is stored: each tile's f is loaded
    // when its processing starts, not with the tile loaded ahead
    load_tile<PREC, VD>(src, g, p, t * kSortTile, min(t * kSortTile + kSortTile, g.n) - 1, ovf, ID);
    // implied cells: the run offsets of a tile's first pass are loaded one
    // tile ahead, and its first run two tiles ahead (the offsets' addresses
    // depend on it), so neither load's latency is waited for when the tile
    // starts
    TbAhead ah{0, 0, 0};
    int b0n = 0;
    if constexpr (IMPL) {
        if (t < ntiles) ah = tile_runs_ahead(g, pv, tile_first_run(pv, t * kSortTile));
        if (t + (int)gridDim.x < ntiles) b0n = tile_first_run(pv, (t + gridDim.x) * kSortTile);
    }
    const int my_tiles = (ntiles - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
    for (; t < ntiles; t += gridDim.x) {
        const int tn = t + gridDim.x;
        prio_by_progress((t - (int)blockIdx.x) / (int)gridDim.x, my_tiles);
        if constexpr (PREC == 1 && !ID) {
            const int last = min(t * kSortTile + kSortTile, g.n) - 1;
#pragma unroll
            for (int k = 0; k < kSortMPT; ++k) p[k].f = src.f[min(t * kSortTile + k * kSortThreads + (int)threadIdx.x, last)];
        }
        if (tn < ntiles)
            load_tile<PREC, VD>(src, g, q, tn * kSortTile, min(tn * kSortTile + kSortTile, g.n) - 1, ovf, ID);
        TbAhead an{0, 0, 0};
        if constexpr (IMPL) {
            const int tnn = tn + gridDim.x;
            if (tn < ntiles) an = tile_runs_ahead(g, pv, b0n);
            if (tnn < ntiles) b0n = tile_first_run(pv, tnn * kSortTile);
        }
        scatter_tile<PREC, VD, PUSH, IMPL, IMPL>(g, sm, p, dst, dtk, bk, offsets, counts, t * kSortTile,
                                                 min(t * kSortTile + kSortTile, g.n) - 1, s_b, fl, pv,
                                                 ovf, s_aux, g.sbins, ah);
#pragma unroll
        for (int k = 0; k < kSortMPT; ++k) p[k] = q[k];
        ah = an;
    }
    if (fl) atomicOr(&s_flags, fl);
    __syncthreads();
    if (threadIdx.x == 0 && s_flags) atomicOr(flags, s_flags);
}

template <int PREC, int VD, bool PUSH, bool IMPL>
__global__ __launch_bounds__(kSortThreads) void k_scatter(Geo g, typename MarkersOf<PREC>::T src,
                                                          typename MarkersOf<PREC>::T dst,
                                                          const double* __restrict__ E,
                                                          const RowShift* __restrict__ rows_g,
                                                          double dtk, float bk,
                                                          const int* __restrict__ offsets,
                                                          int* __restrict__ counts, int* __restrict__ flags, Prev pv)
{
    scatter_tiled<PREC, VD, PUSH, IMPL, true>(g, src, dst, E, rows_g, dtk, bk, offsets, counts, flags, pv);
}

// The step's scatter (push, implied cells, no identities), fitted to five
// waves per SIMD: with the smaller scatter window its LDS admits five blocks
// per CU, and the registers are held to match.
template <int PREC, int VD>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(5)))
void k_scatter_step(Geo g, typename MarkersOf<PREC>::T src, typename MarkersOf<PREC>::T dst,
                    const double* __restrict__ E, const RowShift* __restrict__ rows_g, double dtk, float bk,
                    const int* __restrict__ offsets, int* __restrict__ counts, int* __restrict__ flags, Prev pv)
{
    scatter_tiled<PREC, VD, true, true, false>(g, src, dst, E, rows_g, dtk, bk, offsets, counts, flags, pv);
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
    stage_tables<PREC>(g, sE, sRow, E, rows_g, bk);
    __syncthreads();
    int fl = 0;
    const int base = blockIdx.x * kSortTile;
    for (int k = 0; k < kSortMPT; ++k) {
        int i = base + k * kSortThreads + threadIdx.x;
        if (i < g.n) {
            Pay<PREC, VD> p;
            p.load(m, g, i, true);
            p.push(g, sE, sRow, dtk, bk, fl);
            p.store(m, g, i, true);
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

// Exclusive prefix of the per-tile totals, in place (used when there are too
// many tiles for every block of the apply kernel to sum its predecessors).
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

// Offsets of one tile of kScanTile buckets: the tile's start (the sum of the
// preceding tiles' totals, or an already-scanned prefix when `scanned`) plus
// an in-block exclusive scan of its counts, 16 per thread as 16-byte vectors.
// Also clears the other parity's tile totals for the next count pass, and
// (tfirst non-null) records for every position p = t kTfStride of the new
// order the bucket whose run holds it: tfirst[t].
__device__ __forceinline__ void scan_tile(const int* __restrict__ counts, int nbt, const int* __restrict__ tsum,
                                          int scanned, int* __restrict__ tsum_next, int* __restrict__ offsets,
                                          int tile, int* __restrict__ tfirst)
{
    __shared__ int s_w[kScanThreads / kWave + 1];
    __shared__ int s_pre;
    // the tile's counts first, so their loads overlap the tile-start sum
    const int base = tile * kScanTile + threadIdx.x * kScanItems;
    int c[kScanItems];
    if (base + kScanItems <= nbt) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            const int4 v = *reinterpret_cast<const int4*>(counts + base + k);
            c[k] = v.x; c[k + 1] = v.y; c[k + 2] = v.z; c[k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) c[k] = (base + k < nbt) ? counts[base + k] : 0;
    }
    // tile start
    int pre;
    if (scanned) {
        pre = tsum[tile];
    } else {
        int part = 0;
        for (int t = threadIdx.x; t < tile; t += blockDim.x) part += tsum[t];
        int excl;
        pre = block_excl_scan(part, &excl, s_w);
    }
    if (threadIdx.x == 0) {
        s_pre = pre;
        tsum_next[tile] = 0;
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += c[k];
    int excl;
    block_excl_scan(s, &excl, s_w);
    int run = excl + s_pre;
    int o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = run;
        run += c[k];
    }
    if (tfirst) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            for (int t = (o[k] + kTfStride - 1) >> kTfLog; c[k] > 0 && t <= (o[k] + c[k] - 1) >> kTfLog; ++t)
                tfirst[t] = base + k;
    }
    if (base + kScanItems <= nbt) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4)
            *reinterpret_cast<int4*>(offsets + base + k) = make_int4(o[k], o[k + 1], o[k + 2], o[k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < nbt) offsets[base + k] = o[k];
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int* __restrict__ counts, int nbt,
                                                            const int* __restrict__ tsum, int scanned,
                                                            int* __restrict__ tsum_next, int* __restrict__ offsets,
                                                            int* __restrict__ tfirst)
{
    scan_tile(counts, nbt, tsum, scanned, tsum_next, offsets, blockIdx.x, tfirst);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int PREC>
static size_t sort_smem(const Geo& g, bool push)
{
    (void)push;
    size_t e = sizeof(typename MarkersOf<PREC>::E) * g.nx;
    size_t r = PREC ? sizeof(RowShift) * (g.nv[0] + 1) : 0;
    // the histogram's LDS also holds a tile's implied buckets (FP32 1D-1V)
    const int bins = (PREC == 1 && g.vdim == 1) ? std::max(g.hist_bins, kCountTile) : g.hist_bins;
    return ((e + r + 15) & ~(size_t)15) + sizeof(int) * bins;
}

// LDS of the step's scatter (FP32 1D-1V): a window of at most sbins buckets,
// and a scatter tile's implied buckets.
static size_t scatter_step_smem(const Geo& g)
{
    size_t e = sizeof(float2) * g.nx;
    size_t r = sizeof(RowShift) * (g.nv[0] + 1);
    return ((e + r + 15) & ~(size_t)15) + sizeof(int) * std::max(g.sbins, kSortTile);
}

template <int PREC, int VD>
static hipError_t launch_sort_t(const Geo& g, void* src, void* dst, const double* E, const RowShift* rows,
                                double dtk, float bk, int* counts, int* offsets, int* tile_sums, int* tile_next,
                                int* flags, bool push, hipStream_t st, int phase, const int* off_old,
                                const int* tf_old, int* tf_new)
{
    using MT = typename MarkersOf<PREC>::T;
    MT s = *reinterpret_cast<MT*>(src);
    MT d = dst ? *reinterpret_cast<MT*>(dst) : s;
    // The FP32 1D-1V form uses the tiled count and scatter (one block per
    // resident slot, each walking several tiles; the scatter loads the next
    // while working on the current one) and implied cells when the markers
    // are in a sorted order (off_old); the other forms hold more registers
    // per marker and use one tile per block.
    constexpr bool tiled = PREC == 1 && VD == 1;
    const bool impl = tiled && off_old != nullptr;
    const Prev pv{off_old, tf_old};
    const int ctiles = (g.n + count_tile_size(PREC) - 1) / count_tile_size(PREC);
    const int cblocks = tiled && g.cblocks > 0 ? std::min(ctiles, g.cblocks) : ctiles;
    const int stiles = (g.n + kSortTile - 1) / kSortTile;
    const int sblocks = tiled && g.sblocks > 0 ? std::min(stiles, g.sblocks) : stiles;
    const size_t smem = sort_smem<PREC>(g, push);
    if (g.n == 0 && phase != 1) return hipSuccess;   // the scan still runs: offsets become zero
    static int granted[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    {
        const void* fns[8];
        if constexpr (tiled) {
            fns[0] = (const void*)k_count_tiled<PREC, VD, true, false>;
            fns[1] = (const void*)k_count_tiled<PREC, VD, false, false>;
            fns[2] = (const void*)k_scatter<PREC, VD, true, false>;
            fns[3] = (const void*)k_scatter<PREC, VD, false, false>;
            fns[4] = (const void*)k_count_tiled<PREC, VD, true, true>;
            fns[5] = (const void*)k_count_tiled<PREC, VD, false, true>;
            fns[6] = (const void*)k_scatter<PREC, VD, true, true>;
            fns[7] = (const void*)k_scatter<PREC, VD, false, true>;
        } else {
            fns[0] = fns[4] = (const void*)k_count<PREC, VD, true>;
            fns[1] = fns[5] = (const void*)k_count<PREC, VD, false>;
            fns[2] = fns[6] = (const void*)k_scatter1<PREC, VD, true>;
            fns[3] = fns[7] = (const void*)k_scatter1<PREC, VD, false>;
        }
        for (int i = 0; i < 8; ++i) {
            hipError_t e = ensure_lds(fns[i], smem, granted[i]);
            if (e != hipSuccess) return e;
        }
    }
    const dim3 bl(kSortThreads);
    if (phase == 0) {
        if constexpr (tiled) {
            const dim3 gr(cblocks);
            if (impl) {
                if (push) launch(k_count_tiled<PREC, VD, true, true>, gr, bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags, pv);
                else launch(k_count_tiled<PREC, VD, false, true>, gr, bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags, pv);
            } else {
                if (push) launch(k_count_tiled<PREC, VD, true, false>, gr, bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags, pv);
                else launch(k_count_tiled<PREC, VD, false, false>, gr, bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags, pv);
            }
        } else {
            if (push) launch(k_count<PREC, VD, true>, dim3(cblocks), bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags);
            else launch(k_count<PREC, VD, false>, dim3(cblocks), bl, smem, st, g, s, E, rows, dtk, bk, counts, tile_sums, flags);
        }
    } else if (phase == 1) {
        // tile_sums: this sort's totals; tile_next: the other parity, cleared here
        const int nbt = g.nb + 1;
        const int ntiles = (nbt + kScanTile - 1) / kScanTile;
        int scanned = 0;
        if (ntiles > 1024) {
            hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tile_sums, ntiles);
            scanned = 1;
        }
        hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, st, counts, nbt, tile_sums, scanned,
                           tile_next, offsets, tf_new);
    } else {
        if constexpr (tiled) {
            const dim3 gr(sblocks);
            if (impl) {
                if (push && !s.id) {
                    static int granted_step = 0;
                    const size_t sm_step = scatter_step_smem(g);
                    hipError_t e = ensure_lds((const void*)k_scatter_step<PREC, VD>, sm_step, granted_step);
                    if (e != hipSuccess) return e;
                    launch(k_scatter_step<PREC, VD>, dim3(g.sblocks_step > 0 ? std::min(stiles, g.sblocks_step) : stiles),
                           bl, sm_step, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags, pv);
                } else if (push) launch(k_scatter<PREC, VD, true, true>, gr, bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags, pv);
                else launch(k_scatter<PREC, VD, false, true>, gr, bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags, pv);
            } else {
                if (push) launch(k_scatter<PREC, VD, true, false>, gr, bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags, pv);
                else launch(k_scatter<PREC, VD, false, false>, gr, bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags, pv);
            }
        } else {
            if (push) launch(k_scatter1<PREC, VD, true>, dim3(sblocks), bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags);
            else launch(k_scatter1<PREC, VD, false>, dim3(sblocks), bl, smem, st, g, s, d, E, rows, dtk, bk, offsets, counts, flags);
        }
    }
    return hipGetLastError();
}

// phase 0 = count, 1 = scan, 2 = scatter.  offsets: the run offsets of the new
// order (written by the scan, used by the scatter); off_old / tf_old: the
// order the markers are in, for implied cells (FP32 1D-1V; nullptr when every
// cell index is stored); tf_new (may be null): the scan's record of the new
// order's tile starts.
hipError_t launch_sort(const Geo& g, void* src, void* dst, const double* E, const RowShift* rows,
                       double dtk, float bk, int* counts, int* offsets, int* tile_sums, int* tile_next, int* flags,
                       bool push, hipStream_t st, int phase, const int* off_old, const int* tf_old, int* tf_new)
{
    if (g.prec == 0 && g.vdim == 1) return launch_sort_t<0, 1>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, tile_next, flags, push, st, phase, nullptr, nullptr, tf_new);
    if (g.prec == 0 && g.vdim == 3) return launch_sort_t<0, 3>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, tile_next, flags, push, st, phase, nullptr, nullptr, tf_new);
    if (g.prec == 1 && g.vdim == 1) return launch_sort_t<1, 1>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, tile_next, flags, push, st, phase, off_old, tf_old, tf_new);
    return launch_sort_t<1, 3>(g, src, dst, E, rows, dtk, bk, counts, offsets, tile_sums, tile_next, flags, push, st, phase, nullptr, nullptr, tf_new);
}

// ---------------------------------------------------------------------------
// batched passes: one launch covers every instance of a batch (1D-1V); block b
// belongs to the instance whose prefix range holds b and runs that
// instance's block body with the instance's own geometry and buffers.  The
// instances are always in a sorted order here, so FP32 cells are implied.
// ---------------------------------------------------------------------------
template <int PREC> __device__ __forceinline__ const typename MarkersOf<PREC>::T& bmark(const BInst& I, int b);
template <> __device__ __forceinline__ const M64& bmark<0>(const BInst& I, int b) { return I.m64[b]; }
template <> __device__ __forceinline__ const M32& bmark<1>(const BInst& I, int b) { return I.m32[b]; }

template <int PREC>
__global__ __launch_bounds__(kSortThreads) void k_count_b(const BInst* __restrict__ tab, const int* __restrict__ pre,
                                                          int ninst, int cur)
{
    const int* pr = pre + BPRE_COUNT * (ninst + 1);
    const int i = find_inst(pr, ninst, blockIdx.x);
    const BInst& I = tab[i];
    count_block<PREC, 1, true, PREC == 1>(I.g, bmark<PREC>(I, cur), I.E, I.rows, I.dtk, I.bk, I.counts, I.tsum[cur],
                                          I.flags, blockIdx.x - pr[i], Prev{I.offsets[cur], I.tfirst[cur]});
}

__global__ __launch_bounds__(kScanThreads) void k_scan_b(const BInst* __restrict__ tab, const int* __restrict__ pre,
                                                         int ninst, int cur)
{
    const int* pr = pre + BPRE_SCAN * (ninst + 1);
    const int i = find_inst(pr, ninst, blockIdx.x);
    const BInst& I = tab[i];
    scan_tile(I.counts, I.g.nb + 1, I.tsum[cur], 0, I.tsum[1 - cur], I.offsets[1 - cur], blockIdx.x - pr[i],
              I.tfirst[1 - cur]);
}

template <int PREC>
__global__ __launch_bounds__(kSortThreads) void k_scatter_b(const BInst* __restrict__ tab,
                                                            const int* __restrict__ pre, int ninst, int cur)
{
    const int* pr = pre + BPRE_SCATTER * (ninst + 1);
    const int i = find_inst(pr, ninst, blockIdx.x);
    const BInst& I = tab[i];
    // batch instances carry no marker identities: with the null pointers
    // known at compile time the payload holds no id register
    typename MarkersOf<PREC>::T src = bmark<PREC>(I, cur), dst = bmark<PREC>(I, 1 - cur);
    src.id = nullptr;
    dst.id = nullptr;
    scatter_block<PREC, 1, true, PREC == 1>(I.g, src, dst, I.E, I.rows, I.dtk, I.bk, I.offsets[1 - cur], I.counts,
                                            I.flags, blockIdx.x - pr[i], Prev{I.offsets[cur], I.tfirst[cur]},
                                            PREC == 1 ? I.g.sbins : I.g.hist_bins);
}

// Blocks of a batched pass for one instance (host side).
int sort_blocks(const Geo& g, int phase)
{
    if (phase == 0) return (g.n + count_tile_size(g.prec) - 1) / count_tile_size(g.prec);
    if (phase == 1) return (g.nb + 1 + kScanTile - 1) / kScanTile;
    return (g.n + kSortTile - 1) / kSortTile;
}

// Blocks of the tiled scatter that fit on one CU at once for g's LDS size
// (0 where the form has no tiled scatter); host side.
// Resident blocks per CU of the tiled count pass (FP32 1D-1V) for this
// geometry's LDS; 0 (a tile per block) for the other forms.
int count_blocks_per_cu(const Geo& g)
{
    if (!(g.prec == 1 && g.vdim == 1)) return 0;
    const size_t smem = sort_smem<1>(g, true);
    static int granted = 0;
    int per_cu = 0;
    if (ensure_lds((const void*)k_count_tiled<1, 1, true, true>, smem, granted) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_count_tiled<1, 1, true, true>,
                                                     kSortThreads, smem) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 0;
    }
    return per_cu;
}

int scatter_step_blocks_per_cu(const Geo& g)
{
    if (!(g.prec == 1 && g.vdim == 1)) return 0;
    const size_t smem = scatter_step_smem(g);
    static int granted = 0;
    int per_cu = 0;
    if (ensure_lds((const void*)k_scatter_step<1, 1>, smem, granted) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_scatter_step<1, 1>, kSortThreads,
                                                     smem) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 4;
    }
    return per_cu;
}

int scatter_blocks_per_cu(const Geo& g)
{
    if (!(g.prec == 1 && g.vdim == 1)) return 0;
    const size_t smem = sort_smem<1>(g, true);
    static int granted = 0;
    int per_cu = 0;
    if (ensure_lds((const void*)k_scatter<1, 1, true, true>, smem, granted) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_scatter<1, 1, true, true>, kSortThreads,
                                                     smem) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 4;
    }
    return per_cu;
}

// LDS of the count and scatter blocks for one instance (host side).
size_t sort_lds(const Geo& g) { return g.prec ? sort_smem<1>(g, true) : sort_smem<0>(g, true); }

// LDS of the batched scatter for one instance: the FP32 form's window is the
// step scatter's (sbins buckets), the FP64 form's the count's.
size_t scatter_lds(const Geo& g) { return g.prec ? scatter_step_smem(g) : sort_smem<0>(g, true); }

// phase 0 = count (with push), 1 = scan, 2 = scatter, over `blocks` blocks
hipError_t launch_sort_batch(int prec, const BInst* tab, const int* pre, int ninst, int blocks, size_t smem, int cur,
                             hipStream_t st, int phase)
{
    if (blocks <= 0) return hipSuccess;
    static int granted[4] = {0, 0, 0, 0};
    const void* fns[4] = {(const void*)k_count_b<0>, (const void*)k_count_b<1>, (const void*)k_scatter_b<0>,
                          (const void*)k_scatter_b<1>};
    {
        const int i = (phase == 2 ? 2 : 0) + (prec == 0 ? 0 : 1);
        hipError_t e = phase == 1 ? hipSuccess : ensure_lds(fns[i], smem, granted[i]);
        if (e != hipSuccess) return e;
    }
    const dim3 gr(blocks);
    if (phase == 0) {
        if (prec == 0) hipLaunchKernelGGL(k_count_b<0>, gr, dim3(kSortThreads), smem, st, tab, pre, ninst, cur);
        else hipLaunchKernelGGL(k_count_b<1>, gr, dim3(kSortThreads), smem, st, tab, pre, ninst, cur);
    } else if (phase == 1) {
        hipLaunchKernelGGL(k_scan_b, gr, dim3(kScanThreads), 0, st, tab, pre, ninst, cur);
    } else {
        if (prec == 0) hipLaunchKernelGGL(k_scatter_b<0>, gr, dim3(kSortThreads), smem, st, tab, pre, ninst, cur);
        else hipLaunchKernelGGL(k_scatter_b<1>, gr, dim3(kSortThreads), smem, st, tab, pre, ninst, cur);
    }
    return hipGetLastError();
}

// Stored cell index of every marker of a sorted FP32 1D-1V order: the run a
// position lies in is its cell (the overflow run keeps its stored values).
__global__ __launch_bounds__(256) void k_cells(Geo g, const int* __restrict__ off, int* __restrict__ cell)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < g.nb; b += gridDim.x * blockDim.x) {
        const int lo = off[b], hi = off[b + 1];
        for (int p = lo; p < hi; ++p) cell[p] = b;
    }
}

hipError_t launch_cells(const Geo& g, const int* offsets, int* cell, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const int blocks = std::min((g.nb + 255) / 256, 8192);
    hipLaunchKernelGGL(k_cells, dim3(blocks), dim3(256), 0, st, g, offsets, cell);
    return hipGetLastError();
}

hipError_t launch_push(const Geo& g, void* m, const double* E, const RowShift* rows, double dtk, float bk,
                       int* flags, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const int blocks = (g.n + kSortTile - 1) / kSortTile;
    const size_t smem = (g.prec ? sizeof(float2) : sizeof(double)) * g.nx + (g.prec ? sizeof(RowShift) * (g.nv[0] + 1) : 0);
    if (g.prec == 0 && g.vdim == 1) hipLaunchKernelGGL((k_push<0, 1>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M64*>(m), E, rows, dtk, bk, flags);
    else if (g.prec == 0) hipLaunchKernelGGL((k_push<0, 3>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M64*>(m), E, rows, dtk, bk, flags);
    else if (g.vdim == 1) hipLaunchKernelGGL((k_push<1, 1>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M32*>(m), E, rows, dtk, bk, flags);
    else hipLaunchKernelGGL((k_push<1, 3>), dim3(blocks), dim3(kSortThreads), smem, st, g, *reinterpret_cast<M32*>(m), E, rows, dtk, bk, flags);
    return hipGetLastError();
}

}  // namespace avl
