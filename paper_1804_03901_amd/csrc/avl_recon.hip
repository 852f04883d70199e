// Weight-normalised reconstruction, Eq. (reconstruction), fused with the
// velocity-moment partial sums for rho, for 1D-1V.
//
// Work decomposition.  After the sort, the markers of one dual cell (a "run")
// are contiguous.  A run (i, j) contributes to the four grid cells
// (i, j), (i+1, j), (i, j+1), (i+1, j+1) with weights (1-a)(1-b), a(1-b),
// (1-a)b, ab.  One wavefront owns a strip of 63 target columns and a chunk of
// target rows; lane l owns run column strip*63 - 1 + l.  The wave walks the
// dual rows of its chunk bottom to top: it stages the row segment's markers
// (one contiguous range of the sorted arrays, plus the wrapped run at x = L
// for the first strip) into LDS with coalesced loads, then every lane sums its
// own run into four (N, D) corner partials.  Staging is software-pipelined:
// the next row's markers are loaded into registers while the current row is
// summed, so each wave keeps a full row segment (16-24 KB) of loads in
// flight.  Row segments larger than the LDS capacity are summed straight from
// global memory (same order, slower).  Tasks are dealt to blocks so that each
// XCD gets consecutive chunks of the same strip, whose shared halo rows then
// hit that XCD's L2.  Target cell (i, j) is then
//   ((up01(i, j-1) + up11(i-1, j-1)) + S00(i, j)) + S10(i-1, j)
// where the (i-1) terms come from the neighbouring lane by a shuffle and the
// "up" terms are carried in registers from the previous dual row.  Every sum
// has a fixed order given the sorted input: no float atomics anywhere.
//
// rho: each lane also sums f over the rows of its chunk for its column and
// writes one partial per (chunk, column); the field kernel adds the chunk
// partials in chunk order, in FP64.
#include <type_traits>

#include "avl_device.h"

namespace avl {

template <typename T> struct Kahan {
    T s, c;
    __device__ void zero() { s = T(0); c = T(0); }
    __device__ void add(T x) {
        T y = x - c;
        T t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ T value() const { return s - c; }
};

// Plain FP64 accumulator with the same interface.
struct Plain {
    double s;
    __device__ void zero() { s = 0.0; }
    __device__ void add(double x) { s = s + x; }
    __device__ double value() const { return s; }
};

// Per-run moments of the marker offsets: with them the four cloud-in-cell
// corner sums of a run are
//   N11 = S_abf, N10 = S_af - S_abf, N01 = S_bf - S_abf, N00 = S_f - S_af - S_bf + S_abf
//   D11 = S_ab,  D10 = S_a - S_ab,   D01 = S_b - S_ab,   D00 = n - S_a - S_b + S_ab
// (expanding (1-a)(1-b) etc.), so a marker costs four products and seven
// accumulations instead of eight weighted sums.  The accumulators are FP64
// (A = Plain) or compensated FP32 (A = Kahan<float>).
template <typename A> struct Moments {
    A f, af, bf, abf, a, b, ab;
    __device__ void zero() { f.zero(); af.zero(); bf.zero(); abf.zero(); a.zero(); b.zero(); ab.zero(); }
    template <typename T> __device__ void add(T a_, T b_, T f_) {
        const T af_ = a_ * f_, bf_ = b_ * f_, ab_ = a_ * b_, abf_ = ab_ * f_;
        f.add(f_); af.add(af_); bf.add(bf_); abf.add(abf_);
        a.add(a_); b.add(b_); ab.add(ab_);
    }
};

struct Corners {
    double n00, n10, n01, n11, d00, d10, d01, d11;
    template <typename A> __device__ void from(const Moments<A>& M, int len) {
        const double Sf = M.f.value(), Saf = M.af.value(), Sbf = M.bf.value(), Sabf = M.abf.value();
        const double Sa = M.a.value(), Sb = M.b.value(), Sab = M.ab.value();
        n11 = Sabf;
        n10 = Saf - Sabf;
        n01 = Sbf - Sabf;
        n00 = (Sf - Saf) - n01;
        d11 = Sab;
        d10 = Sa - Sab;
        d01 = Sb - Sab;
        d00 = ((double)len - Sa) - d01;
    }
};


__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int PREC> struct RT;
template <> struct RT<0> {
    using T = double;
    using M = M64;
    static constexpr int KU = 20;    // register prefetch depth per lane (markers)
};
template <> struct RT<1> {
    using T = float;
    using M = M32;
    static constexpr int KU = 20;
};

// LDS capacity per wave: KU markers per lane of the main range plus one
// wrapped run of at most a wavefront.
template <int PREC> constexpr int recon_cap() { return kWave * (RT<PREC>::KU + 1); }

// bytes of LDS per wave: a, b, f as three arrays of the storage type
template <int PREC> constexpr size_t recon_lds() { return 3 * sizeof(typename RT<PREC>::T) * recon_cap<PREC>(); }

// Descriptors cover exactly one range of markers [first, first+count): lanes
// past the end read zero and cost no memory traffic.
template <int PREC> struct Src;
template <> struct Src<0> {           // x, v (first component), f
    __amdgpu_buffer_rsrc_t rx, rv, rf;
    __device__ void init(const M64& m, int first, int count) {
        const size_t b = sizeof(double) * (size_t)count;
        rx = rsrc(m.x + first, b);
        rv = rsrc(m.v + first, b);
        rf = rsrc(m.f + first, b);
    }
    struct Raw { double x, v, f; };
    __device__ Raw load(int byte_off, int soff) const {
        Raw r;
        r.x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, byte_off, soff, 0));
        r.v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, byte_off, soff, 0));
        r.f = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rf, byte_off, soff, 0));
        return r;
    }
};
template <> struct Src<1> {           // a, b (first component), f
    __amdgpu_buffer_rsrc_t ra, rb, rf;
    __device__ void init(const M32& m, int first, int count) {
        const size_t b = sizeof(float) * (size_t)count;
        ra = rsrc(m.a + first, b);
        rb = rsrc(m.b + first, b);
        rf = rsrc(m.f + first, b);
    }
    struct Raw { float a, b, f; };
    __device__ Raw load(int byte_off, int soff) const {
        Raw r;
        r.a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, byte_off, soff, 0));
        r.b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, byte_off, soff, 0));
        r.f = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rf, byte_off, soff, 0));
        return r;
    }
};

// Staged row segment in LDS.  FP32 form: a, b, f as three float arrays
// (12 bytes a marker, so more waves fit per CU).  FP64: (a, b) pairs and f,
// read with one 16-byte and one 8-byte access.
template <int PREC> struct Lds;
template <> struct Lds<1> {
    float *a, *b, *f;
    __device__ void init(unsigned char* base) {
        a = reinterpret_cast<float*>(base);
        b = a + recon_cap<1>();
        f = b + recon_cap<1>();
    }
    __device__ void put(const Geo&, int p, const Src<1>::Raw& r) {
        a[p] = r.a;
        b[p] = r.b;
        f[p] = r.f;
    }
    __device__ void get(int p, float& aa, float& bb, float& ff) const {
        aa = a[p];
        bb = b[p];
        ff = f[p];
    }
};
template <> struct Lds<0> {
    double2* ab;
    double* f;
    __device__ void init(unsigned char* base) {
        ab = reinterpret_cast<double2*>(base);
        f = reinterpret_cast<double*>(base + sizeof(double2) * recon_cap<0>());
    }
    __device__ void put(const Geo& g, int p, const Src<0>::Raw& r) {
        int ix, jp[1];
        double aa, bb[1];
        double vv[1] = {r.v};
        locate64<1>(g, r.x, vv, ix, jp, aa, bb);
        ab[p] = make_double2(aa, bb[0]);
        f[p] = r.f;
    }
    __device__ void get(int p, double& aa, double& bb, double& ff) const {
        const double2 t = ab[p];
        aa = t.x;
        bb = t.y;
        ff = f[p];
    }
};

template <int PREC>
__device__ __forceinline__ void load_global(const Geo& g, const typename RT<PREC>::M& m, int q,
                                            typename RT<PREC>::T& a, typename RT<PREC>::T& b,
                                            typename RT<PREC>::T& f)
{
    if constexpr (PREC == 0) {
        int ix, jp[1];
        double bb[1];
        double vv[1] = {m.v[q]};
        locate64<1>(g, m.x[q], vv, ix, jp, a, bb);
        b = bb[0];
        f = m.f[q];
    } else {
        a = m.a[q];
        b = m.b[q];
        f = m.f[q];
    }
}

// Marker range of one dual-row segment: the contiguous runs of lanes
// first..last plus (first strip only) the wrapped run of lane 0.
struct Seg {
    int lo, nmain, wbeg, wlen;
    __device__ bool fits(int cap_main) const { return nmain <= cap_main && wlen <= kWave; }
};

__device__ __forceinline__ Seg make_seg(int beg, int end, int first_lane, int last_lane, bool wrapped)
{
    Seg s;
    s.lo = __shfl(beg, first_lane, kWave);
    const int hi = __shfl(end, last_lane, kWave);
    s.wbeg = __shfl(beg, 0, kWave);
    const int wend = __shfl(end, 0, kWave);
    s.nmain = hi - s.lo;
    s.wlen = wrapped ? wend - s.wbeg : 0;
    return s;
}

// Issue the loads of one row segment into registers: KU markers per lane of
// the main range and the lane's marker of the wrapped run.  The loads carry
// no branches: each goes through a descriptor bounded to its range.
template <int PREC>
__device__ __forceinline__ void prefetch(const typename RT<PREC>::M& m, const Seg& s, int lane,
                                         typename Src<PREC>::Raw* r, typename Src<PREC>::Raw& w)
{
    constexpr int KU = RT<PREC>::KU;
    constexpr int esz = sizeof(typename RT<PREC>::T);
    if (!s.fits(kWave * KU)) return;   // summed from global memory instead
    Src<PREC> src;
    src.init(m, __builtin_amdgcn_readfirstlane(s.lo), __builtin_amdgcn_readfirstlane(s.nmain));
    const int off = lane * esz;
#pragma unroll
    for (int k = 0; k < KU; ++k) r[k] = src.load(off, k * kWave * esz);
    if (s.wlen) {
        Src<PREC> ws;
        ws.init(m, __builtin_amdgcn_readfirstlane(s.wbeg), __builtin_amdgcn_readfirstlane(s.wlen));
        w = ws.load(off, 0);
    }
}

template <int PREC, bool KAHAN>
__global__ __launch_bounds__(kWave) void k_recon_1v(Geo g, typename RT<PREC>::M m, const int* __restrict__ offsets,
                                                    typename RT<PREC>::T* __restrict__ fgrid,
                                                    typename RT<PREC>::T* __restrict__ Dgrid,
                                                    double* __restrict__ rho_part, int tasks_per_xcd)
{
    using T = typename RT<PREC>::T;
    using A = typename std::conditional<KAHAN, Kahan<float>, Plain>::type;
    constexpr int KU = RT<PREC>::KU;
    constexpr int MAIN = kWave * KU;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    // XCD-aware dealing: blocks go round-robin over the 8 XCDs; give each XCD
    // a contiguous range of (strip-major) tasks
    const int task = (blockIdx.x & 7) * tasks_per_xcd + (blockIdx.x >> 3);
    if ((blockIdx.x >> 3) >= tasks_per_xcd || task >= g.nstrip * g.nchunk) return;
    Lds<PREC> lds;
    lds.init(smem);

    const int strip = task / g.nchunk;
    const int chunk = task - strip * g.nchunk;
    const int nx = g.nx;
    const int col = strip * kReconCols - 1 + lane;        // -1 is the wrapped column nx-1
    const bool run_ok = col < nx;
    const int colw = col < 0 ? nx - 1 : col;
    const bool tgt_ok = lane >= 1 && col < nx;
    const bool wrapped = (strip == 0);
    const int first_lane = wrapped ? 1 : 0;
    const int last_col = min(strip * kReconCols + kReconCols - 1, nx - 1);
    const int last_lane = last_col - (strip * kReconCols - 1);
    const int j_begin = chunk * g.rc;
    const int j_end = min(j_begin + g.rc, g.nv[0]);

    auto row_offsets = [&](int jd, int& beg, int& end) {
        beg = 0;
        end = 0;
        if (run_ok && jd < j_end) {
            const int bk = (jd + 1) * nx + colw;
            beg = offsets[bk];
            end = offsets[bk + 1];
        }
    };

    typename Src<PREC>::Raw regs[KU], wreg;
    int beg, end, nbeg, nend;
    row_offsets(j_begin - 1, beg, end);
    Seg seg = make_seg(beg, end, first_lane, last_lane, wrapped);
    prefetch<PREC>(m, seg, lane, regs, wreg);
    row_offsets(j_begin, nbeg, nend);

    double upN = 0.0, upD = 0.0;
    double rp = 0.0;

    for (int jd = j_begin - 1; jd < j_end; ++jd) {
        const bool staged = seg.fits(MAIN);
        if (staged) {
#pragma unroll
            for (int k = 0; k < KU; ++k) {
                const int p = lane + k * kWave;
                if (p < seg.nmain) lds.put(g, p, regs[k]);
            }
            if (lane < seg.wlen) lds.put(g, seg.nmain + lane, wreg);
        }
        wave_sync_lds();
        const int p0 = staged ? ((wrapped && lane == 0) ? seg.nmain : beg - seg.lo) : beg;
        const int len = end - beg;
        // start the next row's loads before summing this one
        Seg nseg = make_seg(nbeg, nend, first_lane, last_lane, wrapped);
        if (jd + 1 < j_end) prefetch<PREC>(m, nseg, lane, regs, wreg);
        int nnbeg, nnend;
        row_offsets(jd + 2, nnbeg, nnend);

        // Two separate loops: a single loop with a per-iteration choice makes
        // the compiler fall back to generic (flat) loads, whose waits would also
        // stall on the prefetch of the next row.
        Moments<A> M;
        M.zero();
        if (staged) {
            for (int k = 0; k < len; ++k) {
                T a, b, f;
                lds.get(p0 + k, a, b, f);
                if constexpr (KAHAN) M.add(a, b, f);
                else M.add((double)a, (double)b, (double)f);
            }
        } else {
            for (int k = 0; k < len; ++k) {
                T a, b, f;
                load_global<PREC>(g, m, p0 + k, a, b, f);
                if constexpr (KAHAN) M.add(a, b, f);
                else M.add((double)a, (double)b, (double)f);
            }
        }
        wave_sync_lds();
        Corners c;
        c.from(M, len);

        // corner partials of the left neighbour run (lane - 1)
        const double n10l = __shfl_up(c.n10, 1, kWave);
        const double d10l = __shfl_up(c.d10, 1, kWave);
        const double n11l = __shfl_up(c.n11, 1, kWave);
        const double d11l = __shfl_up(c.d11, 1, kWave);

        if (jd >= j_begin && tgt_ok) {
            const double Nv = (upN + c.n00) + n10l;
            const double Dv = (upD + c.d00) + d10l;
            const double fv = Dv > 0.0 ? Nv / Dv : 0.0;
            const size_t gi = (size_t)jd * nx + col;
            fgrid[gi] = (T)fv;
            if (Dgrid) Dgrid[gi] = (T)Dv;
            rp += (double)(T)fv;
        }
        upN = c.n01 + n11l;
        upD = c.d01 + d11l;

        beg = nbeg;
        end = nend;
        nbeg = nnbeg;
        nend = nnend;
        seg = nseg;
    }
    if (tgt_ok) rho_part[(size_t)chunk * nx + col] = rp;
}

hipError_t launch_recon(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid,
                        double* rho_part, hipStream_t st)
{
    if (g.vdim != 1) return hipErrorNotSupported;
    const int tasks = g.nstrip * g.nchunk;
    const int per_xcd = (tasks + 7) / 8;
    const int blocks = per_xcd * 8;
    const size_t smem = g.prec ? recon_lds<1>() : recon_lds<0>();
    static int granted[3] = {0, 0, 0};
    const int var = g.prec == 0 ? 0 : (g.kahan ? 2 : 1);
    const void* fns[3] = {(const void*)k_recon_1v<0, false>, (const void*)k_recon_1v<1, false>,
                          (const void*)k_recon_1v<1, true>};
    hipError_t e = ensure_lds(fns[var], smem, granted[var]);
    if (e != hipSuccess) return e;
    if (var == 0)
        hipLaunchKernelGGL((k_recon_1v<0, false>), dim3(blocks), dim3(kWave), smem, st, g, *reinterpret_cast<M64*>(m),
                           offsets, (double*)fgrid, (double*)Dgrid, rho_part, per_xcd);
    else if (var == 1)
        hipLaunchKernelGGL((k_recon_1v<1, false>), dim3(blocks), dim3(kWave), smem, st, g, *reinterpret_cast<M32*>(m),
                           offsets, (float*)fgrid, (float*)Dgrid, rho_part, per_xcd);
    else
        hipLaunchKernelGGL((k_recon_1v<1, true>), dim3(blocks), dim3(kWave), smem, st, g, *reinterpret_cast<M32*>(m),
                           offsets, (float*)fgrid, (float*)Dgrid, rho_part, per_xcd);
    return hipGetLastError();
}

int recon_capacity(int prec) { return prec ? recon_cap<1>() : recon_cap<0>(); }

}  // namespace avl
