// Weight-normalised reconstruction, Eq. (reconstruction), fused with the
// velocity-moment partial sums for rho, for 1D-1V.
//
// Work decomposition.  After the sort, the markers of one dual cell (a "run")
// are contiguous.  A run (i, j) contributes to the four grid cells
// (i, j), (i+1, j), (i, j+1), (i+1, j+1) with weights (1-a)(1-b), a(1-b),
// (1-a)b, ab.  One wavefront owns a strip of 63 target columns and a chunk of
// target rows; lane l owns run column strip*63 - 1 + l.  The wave walks the
// dual rows of its chunk, upwards for even chunks and downwards for odd ones,
// so that the dual row two neighbouring chunks share is read by both at about
// the same time and the second read hits L2.  For each row it stages the row
// segment's markers (one contiguous range of the sorted arrays, plus the
// wrapped run at x = L for the first strip) into LDS with coalesced loads and
// 16-byte LDS stores, then every lane sums its own run into four (N, D)
// corner partials.  Staging is software-pipelined: the next two rows'
// markers are loaded into registers while the current row is summed.  Row
// segments larger than the LDS capacity are summed straight from global
// memory (same order, slower).  Tasks are dealt to blocks so that each XCD
// gets consecutive chunks of the same strip.  Target cell (i, j) is then
//   ((up01(i, j-1) + up11(i-1, j-1)) + S00(i, j)) + S10(i-1, j)
// in both walk directions, where the (i-1) terms come from the neighbouring
// lane by a shuffle and the terms of the previous dual row of the walk are
// carried in registers.  A run's own sums do not depend on the order of its
// markers (FixGrid in avl_device.h), and everything above them is added in a
// fixed order, so the grid is a function of the marker multiset alone: no
// float atomics anywhere.
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

// Per-run moments of the marker offsets: with them the four cloud-in-cell
// corner sums of a run are
//   N11 = S_abf, N10 = S_af - S_abf, N01 = S_bf - S_abf, N00 = S_f - S_af - S_bf + S_abf
//   D11 = S_ab,  D10 = S_a - S_ab,   D01 = S_b - S_ab,   D00 = n - S_a - S_b + S_ab
// (expanding (1-a)(1-b) etc.), so a marker costs four products and seven
// accumulations instead of eight weighted sums.  The accumulators are FP64
// and order-independent (FixGrid in avl_device.h): S_f, S_af, S_bf and S_abf
// on a grid fitted to the run's largest |f|, S_a, S_b and S_ab on the grid of
// a run whose largest f is 1 (their terms lie in [0, 1)).
struct FixMoments {
    double f, af, bf, abf, a, b, ab;
    double Cf, Cd;
    __device__ void init(const FixGrid& gf, const FixGrid& gd) {
        Cf = gf.C;
        Cd = gd.C;
        f = af = bf = abf = Cf;
        a = b = ab = Cd;
    }
    // FP64 rounding toward -infinity: each operation adds floor(term / q) q
    __device__ void add_rd(double a_, double b_, double f_) {
        const double ab_ = a_ * b_;
        f += f_;
        a += a_;
        b += b_;
        af = fma(a_, f_, af);
        bf = fma(b_, f_, bf);
        ab = fma(a_, b_, ab);
        abf = fma(ab_, f_, abf);
    }
    // default rounding: each term is rounded down onto its grid explicitly
    __device__ void add_floor(const FixGrid& gf, const FixGrid& gd, double a_, double b_, double f_) {
        const double ab_ = a_ * b_;
        f += fixsum_floor(gf, f_);
        a += fixsum_floor(gd, a_);
        b += fixsum_floor(gd, b_);
        af += fixsum_floor(gf, a_ * f_);
        bf += fixsum_floor(gf, b_ * f_);
        ab += fixsum_floor(gd, ab_);
        abf += fixsum_floor(gf, ab_ * f_);
    }
    __device__ void pin() {
        fixsum_pin(f); fixsum_pin(af); fixsum_pin(bf); fixsum_pin(abf);
        fixsum_pin(a); fixsum_pin(b); fixsum_pin(ab);
    }
};

// Compensated FP32 corner sums (the AVL_OPT_KAHAN32 form): the four corner
// weights (1-a)(1-b), a(1-b), (1-a)b, ab are formed per marker and N and D of
// each corner are summed directly.  Every term is non-negative for f >= 0, so
// no corner is a difference of larger sums: a corner whose weights are all
// small keeps its own relative accuracy.
struct CornerKahan32 {
    Kahan<float> n00, n10, n01, n11, d00, d10, d01, d11;
    __device__ void zero() {
        n00.zero(); n10.zero(); n01.zero(); n11.zero();
        d00.zero(); d10.zero(); d01.zero(); d11.zero();
    }
    __device__ void add(float a_, float b_, float f_) {
        const float oa = 1.0f - a_, ob = 1.0f - b_;
        const float w00 = oa * ob, w10 = a_ * ob, w01 = oa * b_, w11 = a_ * b_;
        n00.add(w00 * f_); n10.add(w10 * f_); n01.add(w01 * f_); n11.add(w11 * f_);
        d00.add(w00); d10.add(w10); d01.add(w01); d11.add(w11);
    }
};

struct Corners {
    double n00, n10, n01, n11, d00, d10, d01, d11;
    __device__ void from(const FixMoments& M, int len) {
        set(M.f - M.Cf, M.af - M.Cf, M.bf - M.Cf, M.abf - M.Cf, M.a - M.Cd, M.b - M.Cd, M.ab - M.Cd, len);
    }
    __device__ void from(const CornerKahan32& K) {
        n00 = K.n00.value(); n10 = K.n10.value(); n01 = K.n01.value(); n11 = K.n11.value();
        d00 = K.d00.value(); d10 = K.d10.value(); d01 = K.d01.value(); d11 = K.d11.value();
    }
    __device__ void set(double Sf, double Saf, double Sbf, double Sabf, double Sa, double Sb, double Sab, int len) {
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


// Lane l receives lane l-1's value (lane 0 receives 0): a DPP shift of the
// whole wavefront by one lane, two 32-bit moves for a double.
__device__ __forceinline__ double from_left(double v)
{
    constexpr int kWaveShr1 = 0x138;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kWaveShr1, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kWaveShr1, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Largest and smallest of a value over the wavefront: DPP steps within quads,
// half rows and rows of 16 lanes, then row broadcasts, leave the result in
// lane 63.  Lanes a step does not write take the identity (0 for the maximum,
// all ones for the minimum).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));   // quad_perm 2,3,0,1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));  // row_mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v)
{
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0xb1, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4e, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x141, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x140, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xa, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int PREC> struct RT;
template <> struct RT<0> {
    using T = double;
    using M = M64;
    // register prefetch depth per lane (markers); 18 keeps the staging buffer
    // at 29 KB, so five waves fit in a compute unit's LDS
    static constexpr int KU = 18;
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
    // V consecutive markers as one 16-byte load per array
    static constexpr int V = 2;
    struct Vec { Raw r[V]; };
    __device__ Vec loadv(int byte_off, int soff) const {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(rx, byte_off, soff, 0);
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rv, byte_off, soff, 0);
        const auto f = __builtin_amdgcn_raw_buffer_load_b128(rf, byte_off, soff, 0);
        const unsigned x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
        const unsigned v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
        const unsigned f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3];
        Vec o;
        o.r[0].x = __hiloint2double((int)x1, (int)x0);
        o.r[1].x = __hiloint2double((int)x3, (int)x2);
        o.r[0].v = __hiloint2double((int)v1, (int)v0);
        o.r[1].v = __hiloint2double((int)v3, (int)v2);
        o.r[0].f = __hiloint2double((int)f1, (int)f0);
        o.r[1].f = __hiloint2double((int)f3, (int)f2);
        return o;
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
    // V consecutive markers as one 16-byte load per array
    static constexpr int V = 4;
    struct Vec { Raw r[V]; };
    __device__ Vec loadv(int byte_off, int soff) const {
        const auto a = __builtin_amdgcn_raw_buffer_load_b128(ra, byte_off, soff, 0);
        const auto b = __builtin_amdgcn_raw_buffer_load_b128(rb, byte_off, soff, 0);
        const auto f = __builtin_amdgcn_raw_buffer_load_b128(rf, byte_off, soff, 0);
        Vec o;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            // elements taken as values first (a bit cast of a vector element
            // subscript reads element 0)
            const unsigned ua = a[q], ub = b[q], uf = f[q];
            o.r[q].a = __uint_as_float(ua);
            o.r[q].b = __uint_as_float(ub);
            o.r[q].f = __uint_as_float(uf);
        }
        return o;
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
    // V = 4 consecutive markers from p (a multiple of 4) as 16-byte stores
    __device__ void putv(const Geo&, int p, const Src<1>::Vec& v) {
        *reinterpret_cast<float4*>(a + p) = make_float4(v.r[0].a, v.r[1].a, v.r[2].a, v.r[3].a);
        *reinterpret_cast<float4*>(b + p) = make_float4(v.r[0].b, v.r[1].b, v.r[2].b, v.r[3].b);
        *reinterpret_cast<float4*>(f + p) = make_float4(v.r[0].f, v.r[1].f, v.r[2].f, v.r[3].f);
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
    __device__ void putv(const Geo& g, int p, const Src<0>::Vec& v) {
#pragma unroll
        for (int q = 0; q < Src<0>::V; ++q) put(g, p + q, v.r[q]);
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
    // the lanes are wave-uniform: scalar reads of one lane each
    s.lo = __builtin_amdgcn_readlane(beg, first_lane);
    const int hi = __builtin_amdgcn_readlane(end, last_lane);
    s.wbeg = __builtin_amdgcn_readlane(beg, 0);
    const int wend = __builtin_amdgcn_readlane(end, 0);
    s.nmain = hi - s.lo;
    s.wlen = wrapped ? wend - s.wbeg : 0;
    return s;
}

// Issue the loads of one row segment into registers: KU markers per lane of
// the main range, V consecutive markers per 16-byte load (lane l takes
// markers u*64*V + l*V + q), and the lane's marker of the wrapped run.  The
// loads carry no branches: each goes through a descriptor bounded to its
// range (rounded up to whole vectors; the few markers read past a segment lie
// inside the marker buffer and are never staged), and a segment that does
// not fit is given an empty range, so all its loads return zero.
// SPARSE (rows well below the register capacity): loads of whole vectors past
// the segment are not issued at all (a wave-uniform test per vector); their
// registers keep stale values that are never staged.
template <int PREC, bool SPARSE = false>
__device__ __forceinline__ void prefetch(const typename RT<PREC>::M& m, const Seg& s, int lane,
                                         typename Src<PREC>::Vec* r, typename Src<PREC>::Raw& w)
{
    constexpr int KU = RT<PREC>::KU;
    constexpr int V = Src<PREC>::V;
    constexpr int esz = sizeof(typename RT<PREC>::T);
    const bool fit = s.fits(kWave * KU);
    const int lo = __builtin_amdgcn_readfirstlane(s.lo);
    const int nm = __builtin_amdgcn_readfirstlane(fit ? (s.nmain + V - 1) / V * V : 0);
    Src<PREC> src;
    src.init(m, lo, nm);
    const int off = lane * V * esz;
#pragma unroll
    for (int u = 0; u < KU / V; ++u) {
        if (SPARSE && u * kWave * V >= nm) break;
        r[u] = src.loadv(off, u * kWave * V * esz);
    }
    // the wrapped run exists for the first strip only (a wave-uniform test)
    const int wl = __builtin_amdgcn_readfirstlane(fit ? s.wlen : 0);
    if (wl > 0) {
        Src<PREC> ws;
        ws.init(m, __builtin_amdgcn_readfirstlane(s.wbeg), wl);
        w = ws.load(lane * esz, 0);
    }
}

// Register prefetch depth: rows of markers in flight per wave while one row
// is summed.  The FP32 form holds two rows ahead (its rows take 60 registers);
// the FP64 form one.
template <int PREC> constexpr int recon_depth() { return PREC ? 2 : 1; }

template <int PREC, bool KAHAN, bool SPARSE, bool PRIO = false>
__device__ __forceinline__ void recon_task(const Geo& g, const typename RT<PREC>::M& m,
                                           const int* __restrict__ offsets, typename RT<PREC>::T* __restrict__ fgrid,
                                           typename RT<PREC>::T* __restrict__ Dgrid, double* __restrict__ rho_part,
                                           int task)
{
    using T = typename RT<PREC>::T;
    using Raw = typename Src<PREC>::Raw;
    using Vec = typename Src<PREC>::Vec;
    constexpr int V = Src<PREC>::V;
    constexpr int KU = RT<PREC>::KU;
    constexpr int MAIN = kWave * KU;
    constexpr int DEPTH = recon_depth<PREC>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
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
    // the chunk walks dual rows j_begin-1 .. j_end-1, upwards for even chunks
    // and downwards for odd ones: the dual row two neighbouring chunks share
    // is then read by both at about the same time (both first or both last),
    // so the second read tends to hit the XCD's L2
    const int nrows = j_end - j_begin + 1;
    const bool upward = (chunk & 1) == 0;

    // run bounds through a bounded descriptor: an invalid lane or row reads
    // past the end and gets (0, 0), with no branch
    const __amdgpu_buffer_rsrc_t roff = rsrc(offsets, sizeof(int) * ((size_t)g.nb + 2));
    auto row_offsets = [&](int k, int& beg, int& end) {
        const bool ok = run_ok && k < nrows;
        const int bk = ok ? (upward ? j_begin + k : j_end - k) * nx + colw : g.nb + 2;
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(roff, bk * (int)sizeof(int), 0, 0);
        const unsigned t0 = t[0], t1 = t[1];
        beg = (int)t0;
        end = (int)t1;
    };

    // Pipeline state: the lane's run bounds and the segment of the current
    // row (k) and of the rows already in flight, and the run bounds of the
    // row whose loads are issued next.
    Vec regs[DEPTH][KU / V];
    Raw wreg[DEPTH];
    int rb[DEPTH + 2], re[DEPTH + 2];
    Seg sg[DEPTH + 1];
#pragma unroll
    for (int q = 0; q < DEPTH + 1; ++q) row_offsets(q, rb[q], re[q]);
#pragma unroll
    for (int q = 0; q < DEPTH; ++q) {
        sg[q] = make_seg(rb[q], re[q], first_lane, last_lane, wrapped);
        prefetch<PREC, SPARSE>(m, sg[q], lane, regs[q], wreg[q]);
    }

    // carried from the previous row of the walk: the up terms (upward) or
    // the 00 term and the left neighbour's 10 term (downward)
    double cN = 0.0, cD = 0.0, cN10 = 0.0, cD10 = 0.0;
    double rp = 0.0;

    // one row of the walk; its markers are in regs[buf]
    auto row = [&](int k, Vec* R, Raw& W) {
        const int tj = upward ? j_begin - 1 + k : j_end - k;   // target row completed by this row
        const Seg seg = sg[0];
        const int beg = rb[0], end = re[0];
        const bool staged = seg.fits(MAIN);
        // order-free bounds of the staged segment: the largest |f| and the
        // smallest nonzero |f| (magnitude bits) over its markers; the minimum
        // is kept as min(k - 1), which a zero key (wrapping to the largest
        // value) cannot lower
        unsigned smax = 0u, smin1 = ~0u;
        if (staged) {
#pragma unroll
            for (int u = 0; u < KU / V; ++u) {
                if (SPARSE && u * kWave * V >= seg.nmain) break;     // not loaded (wave-uniform)
                lds.putv(g, u * kWave * V + lane * V, R[u]);
                if constexpr (!KAHAN) {
                    const int left = seg.nmain - (u * kWave * V + lane * V);   // markers of the vector in range
#pragma unroll
                    for (int q = 0; q < V; ++q) {
                        const unsigned kf = q < left ? fix_key((T)R[u].r[q].f) : 0u;
                        smax = max(smax, kf);
                        smin1 = min(smin1, kf - 1u);
                    }
                }
            }
            // slots past the main range hold zeros from the bounded loads;
            // the wrapped run is written over them afterwards
            if (lane < seg.wlen) {
                lds.put(g, seg.nmain + lane, W);
                const unsigned kf = fix_key((T)W.f);
                smax = max(smax, kf);
                smin1 = min(smin1, kf - 1u);
            }
        }
        wave_sync_lds();
        const int p0 = staged ? ((wrapped && lane == 0) ? seg.nmain : beg - seg.lo) : beg;
        const int len = end - beg;
        // fetch the run bounds of row k+DEPTH+1, then refill the buffer just
        // staged with row k+DEPTH (an empty range past the last row).  The
        // bounds load goes first: loads complete in issue order, so waiting
        // for it later must not also wait for this prefetch.
        row_offsets(k + DEPTH + 1, rb[DEPTH + 1], re[DEPTH + 1]);
        sg[DEPTH] = make_seg(rb[DEPTH], re[DEPTH], first_lane, last_lane, wrapped);
        prefetch<PREC, SPARSE>(m, sg[DEPTH], lane, R, W);

        // Separate loops for staged and global rows: a single loop with a
        // per-iteration choice makes the compiler fall back to generic (flat)
        // loads, whose waits would also stall on the prefetch of the next rows.
        Corners c;
        if constexpr (KAHAN) {
            CornerKahan32 K;
            K.zero();
            if (staged) {
                for (int u = 0; u < len; ++u) {
                    T a, b, f;
                    lds.get(p0 + u, a, b, f);
                    K.add(a, b, f);
                }
            } else {
                for (int u = 0; u < len; ++u) {
                    T a, b, f;
                    load_global<PREC>(g, m, p0 + u, a, b, f);
                    K.add(a, b, f);
                }
            }
            c.from(K);
        } else {
            // the run's grids from order-free bounds: its largest |f| and its
            // length.  The offset sums take the grid of terms below 2^1 (the
            // largest weight, 1, taken as f = 1): for f = c = 2^k on every
            // marker the f grid is then c times the offset grid, every N sum is
            // c times its D sum, and f = c comes out exactly
            //
            // A staged segment whose nonzero |f| all share one binary exponent
            // or two (a factor below 4, as along x in a smooth distribution)
            // takes the segment's largest |f| as every run's bound: each run's
            // own largest |f| is at least the segment's smallest, so its grid is
            // at most twice as coarse as its own bound would give, and the pass
            // over the run is saved.  Otherwise each run takes its own bound.
            unsigned kmax = 0;
            bool narrow = false;
            if (staged) {
                const unsigned gmax = wave_max_u32(smax), gmin = wave_min_u32(smin1) + 1u;
                narrow = gmax == 0u || fix_exp_of_key(gmax, T()) - fix_exp_of_key(gmin, T()) <= 1;
                if (narrow) kmax = gmax;
            }
            if (!narrow) {
                if (staged) {
                    for (int u = 0; u < len; ++u) kmax = max(kmax, fix_key(lds.f[p0 + u]));
                } else {
                    for (int u = 0; u < len; ++u) kmax = max(kmax, fix_key(m.f[p0 + u]));
                }
            }
            const int emax = len > 0 ? fix_exp_of_key(kmax, T()) : -1100;
            const FixGrid gf = fix_grid(emax, len), gd = fix_grid(0, len);
            FixMoments M;
            M.init(gf, gd);
            if (staged) {
                fixsum_round_down();
                M.pin();
                for (int u = 0; u < len; ++u) {
                    T a, b, f;
                    lds.get(p0 + u, a, b, f);
                    M.add_rd((double)a, (double)b, (double)f);
                }
                M.pin();
                fixsum_round_nearest();
                M.pin();
            } else {
                // the FP64 form locates each marker here, in the default rounding
                for (int u = 0; u < len; ++u) {
                    T a, b, f;
                    load_global<PREC>(g, m, p0 + u, a, b, f);
                    M.add_floor(gf, gd, (double)a, (double)b, (double)f);
                }
            }
            c.from(M, len);
        }
        wave_sync_lds();

        // corner partials of the left neighbour run (lane - 1)
        const double n10l = from_left(c.n10);
        const double d10l = from_left(c.d10);
        const double n11l = from_left(c.n11);
        const double d11l = from_left(c.d11);

        // target row j = ((up01 + up11 of dual row j-1) + down00) + down10 of
        // dual row j, in this order in both walk directions
        const double uN = c.n01 + n11l, uD = c.d01 + d11l;
        if (k > 0 && k < nrows && tgt_ok) {
            const double Nv = upward ? (cN + c.n00) + n10l : (uN + cN) + cN10;
            const double Dv = upward ? (cD + c.d00) + d10l : (uD + cD) + cD10;
            const double fv = Dv > 0.0 ? Nv / Dv : 0.0;
            const size_t gi = (size_t)tj * nx + col;
            fgrid[gi] = (T)fv;
            if (Dgrid) Dgrid[gi] = (T)Dv;
            rp += (double)(T)fv;
        }
        cN = upward ? uN : c.n00;
        cD = upward ? uD : c.d00;
        cN10 = n10l;
        cD10 = d10l;

#pragma unroll
        for (int q = 0; q < DEPTH; ++q) sg[q] = sg[q + 1];
#pragma unroll
        for (int q = 0; q < DEPTH + 1; ++q) {
            rb[q] = rb[q + 1];
            re[q] = re[q + 1];
        }
    };

    // whole groups of DEPTH rows, so every pass of the loop body is the same
    // (the compiler then keeps the waits for loads at their full depth); a
    // row past the chunk has empty runs and writes nothing
    // PRIO: issue priority from progress (one instance's tasks, all of about
    // the same size; the batched kernel's tasks differ too much for it)
    for (int k = 0; k < nrows; k += DEPTH) {
        if constexpr (PRIO) prio_by_progress(k, nrows);
#pragma unroll
        for (int q = 0; q < DEPTH; ++q) row(k + q, regs[q], wreg[q]);
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    if (tgt_ok) rho_part[(size_t)chunk * nx + col] = rp;
}

// XCD-aware dealing: blocks go round-robin over the 8 XCDs; give each XCD a
// contiguous range of (strip-major) tasks.  Returns -1 past the last task.
__device__ __forceinline__ int dealt_task(int tasks_per_xcd, int ntask)
{
    const int task = (blockIdx.x & 7) * tasks_per_xcd + (blockIdx.x >> 3);
    return ((blockIdx.x >> 3) >= tasks_per_xcd || task >= ntask) ? -1 : task;
}

template <int PREC, bool KAHAN, bool SPARSE>
__global__ __launch_bounds__(kWave) void k_recon_1v(Geo g, typename RT<PREC>::M m, const int* __restrict__ offsets,
                                                    typename RT<PREC>::T* __restrict__ fgrid,
                                                    typename RT<PREC>::T* __restrict__ Dgrid,
                                                    double* __restrict__ rho_part, int tasks_per_xcd)
{
    const int task = dealt_task(tasks_per_xcd, g.nstrip * g.nchunk);
    if (task < 0) return;
    recon_task<PREC, KAHAN, SPARSE, true>(g, m, offsets, fgrid, Dgrid, rho_part, task);
}

// Batched reconstruction: the tasks of every instance form one list, dealt
// over the XCDs as above; a task runs with its instance's geometry.
template <int PREC> __device__ __forceinline__ const typename RT<PREC>::M& rmark(const BInst& I, int b);
template <> __device__ __forceinline__ const M64& rmark<0>(const BInst& I, int b) { return I.m64[b]; }
template <> __device__ __forceinline__ const M32& rmark<1>(const BInst& I, int b) { return I.m32[b]; }

template <int PREC, bool KAHAN, bool SPARSE>
__global__ __launch_bounds__(kWave) void k_recon_b(const BInst* __restrict__ tab, const int* __restrict__ pre,
                                                   int ninst, int cur, int tasks_per_xcd)
{
    const int* pr = pre + BPRE_RECON * (ninst + 1);
    const int task = dealt_task(tasks_per_xcd, pr[ninst]);
    if (task < 0) return;
    const int i = find_inst(pr, ninst, task);
    const BInst& I = tab[i];
    recon_task<PREC, KAHAN, SPARSE>(I.g, rmark<PREC>(I, cur), I.offsets[cur], (typename RT<PREC>::T*)I.fgrid, nullptr,
                            I.rho_part, task - pr[i]);
}

// Rows of the FP32 form well below the register capacity (on average at most
// 60% of it, e.g. 8 markers a cell) take the SPARSE kernels: at 8 markers a
// cell they are 8-10% faster, at 16 about as fast as the dense ones.
bool recon_sparse(const Geo& g)
{
    if (g.prec != 1 || g.nb <= 0) return false;
    if (g.rform) return g.rform == 2;
    const double per_row = (double)g.n / (double)g.nb * kReconCols;
    return per_row <= 0.6 * kWave * RT<1>::KU;
}

hipError_t launch_recon_batch(int prec, int kahan, int sparse, const BInst* tab, const int* pre, int ninst, int tasks,
                              int cur, hipStream_t st)
{
    if (tasks <= 0) return hipSuccess;
    const int per_xcd = (tasks + 7) / 8;
    const int blocks = per_xcd * 8;
    const size_t smem = prec ? recon_lds<1>() : recon_lds<0>();
    static int granted[5] = {0, 0, 0, 0, 0};
    const int var = prec == 0 ? 0 : 1 + (kahan ? 1 : 0) + (sparse ? 2 : 0);
    const void* fns[5] = {(const void*)k_recon_b<0, false, false>, (const void*)k_recon_b<1, false, false>,
                          (const void*)k_recon_b<1, true, false>, (const void*)k_recon_b<1, false, true>,
                          (const void*)k_recon_b<1, true, true>};
    hipError_t e = ensure_lds(fns[var], smem, granted[var]);
    if (e != hipSuccess) return e;
    const dim3 gr(blocks), bl(kWave);
    switch (var) {
    case 0: hipLaunchKernelGGL((k_recon_b<0, false, false>), gr, bl, smem, st, tab, pre, ninst, cur, per_xcd); break;
    case 1: hipLaunchKernelGGL((k_recon_b<1, false, false>), gr, bl, smem, st, tab, pre, ninst, cur, per_xcd); break;
    case 2: hipLaunchKernelGGL((k_recon_b<1, true, false>), gr, bl, smem, st, tab, pre, ninst, cur, per_xcd); break;
    case 3: hipLaunchKernelGGL((k_recon_b<1, false, true>), gr, bl, smem, st, tab, pre, ninst, cur, per_xcd); break;
    default: hipLaunchKernelGGL((k_recon_b<1, true, true>), gr, bl, smem, st, tab, pre, ninst, cur, per_xcd); break;
    }
    return hipGetLastError();
}

hipError_t launch_recon(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid,
                        double* rho_part, hipStream_t st)
{
    if (g.vdim != 1) return hipErrorNotSupported;
    const int tasks = g.nstrip * g.nchunk;
    const int per_xcd = (tasks + 7) / 8;
    const int blocks = per_xcd * 8;
    const size_t smem = g.prec ? recon_lds<1>() : recon_lds<0>();
    static int granted[5] = {0, 0, 0, 0, 0};
    const int var = g.prec == 0 ? 0 : 1 + (g.kahan ? 1 : 0) + (recon_sparse(g) ? 2 : 0);
    const void* fns[5] = {(const void*)k_recon_1v<0, false, false>, (const void*)k_recon_1v<1, false, false>,
                          (const void*)k_recon_1v<1, true, false>, (const void*)k_recon_1v<1, false, true>,
                          (const void*)k_recon_1v<1, true, true>};
    hipError_t e = ensure_lds(fns[var], smem, granted[var]);
    if (e != hipSuccess) return e;
    const dim3 gr(blocks), bl(kWave);
    if (var == 0) {
        launch(k_recon_1v<0, false, false>, gr, bl, smem, st, g, *reinterpret_cast<M64*>(m), offsets, (double*)fgrid,
               (double*)Dgrid, rho_part, per_xcd);
        return hipGetLastError();
    }
    const M32 m32 = *reinterpret_cast<M32*>(m);
    float* fg = (float*)fgrid;
    float* Dg = (float*)Dgrid;
    switch (var) {
    case 1: launch(k_recon_1v<1, false, false>, gr, bl, smem, st, g, m32, offsets, fg, Dg, rho_part, per_xcd); break;
    case 2: launch(k_recon_1v<1, true, false>, gr, bl, smem, st, g, m32, offsets, fg, Dg, rho_part, per_xcd); break;
    case 3: launch(k_recon_1v<1, false, true>, gr, bl, smem, st, g, m32, offsets, fg, Dg, rho_part, per_xcd); break;
    default: launch(k_recon_1v<1, true, true>, gr, bl, smem, st, g, m32, offsets, fg, Dg, rho_part, per_xcd); break;
    }
    return hipGetLastError();
}

int recon_capacity(int prec) { return prec ? recon_cap<1>() : recon_cap<0>(); }

// Reconstruction waves resident per compute unit, from the occupancy query:
// two per SIMD by the register budget, fewer where a compute unit's LDS holds
// fewer staging buffers (the FP64 form's 29 KB a wave: five).  Without a device,
// the LDS arithmetic on lds_per_cu bytes.
int recon_waves_per_cu(int prec, int lds_per_cu)
{
    const size_t per_wave = prec ? recon_lds<1>() : recon_lds<0>();
    const void* fn = prec ? (const void*)k_recon_1v<1, false, false> : (const void*)k_recon_1v<0, false, false>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave, per_wave) != hipSuccess || per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (size_t)lds_per_cu / per_wave));
    }
    return per_cu;
}

}  // namespace avl
