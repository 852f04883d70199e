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
// own run into four (N, D) corner partials.  Target cell (i, j) is then
//   ((up01(i, j-1) + up11(i-1, j-1)) + S00(i, j)) + S10(i-1, j)
// where the (i-1) terms come from the neighbouring lane by a shuffle and the
// "up" terms are carried in registers from the previous dual row.  Every sum
// has a fixed order given the sorted input: no float atomics anywhere.
//
// rho: each lane also sums f over the rows of its chunk for its column and
// writes one partial per (chunk, column); the field kernel adds the chunk
// partials in chunk order, in FP64.
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

template <int PREC> struct ReconTypes;
template <> struct ReconTypes<0> { using T = double; using Acc = Plain; using M = M64; };
template <> struct ReconTypes<1> { using T = float; using Acc = Kahan<float>; using M = M32; };

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int PREC>
__device__ __forceinline__ void load_ab(const Geo& g, const typename ReconTypes<PREC>::M& m, int q,
                                        typename ReconTypes<PREC>::T& a, typename ReconTypes<PREC>::T& b,
                                        typename ReconTypes<PREC>::T& f);

template <>
__device__ __forceinline__ void load_ab<0>(const Geo& g, const M64& m, int q, double& a, double& b, double& f)
{
    int ix, jp[1];
    double bb[1];
    double vv[1] = {m.v[q]};
    locate64<1>(g, m.x[q], vv, ix, jp, a, bb);
    b = bb[0];
    f = m.f[q];
}

template <>
__device__ __forceinline__ void load_ab<1>(const Geo& g, const M32& m, int q, float& a, float& b, float& f)
{
    a = m.a[q];
    b = m.b[q];
    f = m.f[q];
}

template <int PREC>
__global__ __launch_bounds__(kWave * kReconWaves) void k_recon_1v(Geo g, typename ReconTypes<PREC>::M m,
                                                                  const int* __restrict__ offsets,
                                                                  typename ReconTypes<PREC>::T* __restrict__ fgrid,
                                                                  typename ReconTypes<PREC>::T* __restrict__ Dgrid,
                                                                  double* __restrict__ rho_part)
{
    using T = typename ReconTypes<PREC>::T;
    using Acc = typename ReconTypes<PREC>::Acc;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int task = blockIdx.x * kReconWaves + wv;
    if (task >= g.nstrip * g.nchunk) return;
    T* sA = reinterpret_cast<T*>(smem) + (size_t)wv * 3 * g.cap;
    T* sB = sA + g.cap;
    T* sF = sB + g.cap;

    const int strip = task % g.nstrip;
    const int chunk = task / g.nstrip;
    const int nx = g.nx;
    const int col = strip * kReconCols - 1 + lane;        // -1 .. ; -1 is the wrapped column nx-1
    const bool run_ok = col < nx;
    const int colw = col < 0 ? nx - 1 : col;
    const bool tgt_ok = lane >= 1 && col < nx;
    const bool wrapped = (strip == 0);
    const int first_lane = wrapped ? 1 : 0;
    const int last_col = min(strip * kReconCols + kReconCols - 1, nx - 1);
    const int last_lane = last_col - (strip * kReconCols - 1);
    const int j_begin = chunk * g.rc;
    const int j_end = min(j_begin + g.rc, g.nv[0]);

    Acc upN, upD;
    upN.zero();
    upD.zero();
    double rp = 0.0;

    for (int jd = j_begin - 1; jd < j_end; ++jd) {
        const int rowbase = (jd + 1) * nx;
        int beg = 0, end = 0;
        if (run_ok) {
            beg = offsets[rowbase + colw];
            end = offsets[rowbase + colw + 1];
        }
        const int lo = __shfl(beg, first_lane, kWave);
        const int hi = __shfl(end, last_lane, kWave);
        const int wbeg = __shfl(beg, 0, kWave);
        const int wend = __shfl(end, 0, kWave);
        const int nmain = hi - lo;
        const int total = nmain + (wrapped ? wend - wbeg : 0);
        const bool staged = total <= g.cap;
        int p0;
        if (staged) {
            for (int p = lane; p < total; p += kWave) {
                int q = p < nmain ? lo + p : wbeg + (p - nmain);
                T a, b, f;
                load_ab<PREC>(g, m, q, a, b, f);
                sA[p] = a;
                sB[p] = b;
                sF[p] = f;
            }
            wave_sync_lds();
            p0 = (wrapped && lane == 0) ? nmain : beg - lo;
        } else {
            p0 = beg;
        }
        const int len = end - beg;

        Acc n00, n10, n01, n11, d00, d10, d01, d11;
        n00.zero(); n10.zero(); n01.zero(); n11.zero();
        d00.zero(); d10.zero(); d01.zero(); d11.zero();
        for (int k = 0; k < len; ++k) {
            T a, b, f;
            if (staged) {
                a = sA[p0 + k];
                b = sB[p0 + k];
                f = sF[p0 + k];
            } else {
                load_ab<PREC>(g, m, p0 + k, a, b, f);
            }
            const T ua = T(1) - a, ub = T(1) - b;
            const T w00 = ua * ub, w10 = a * ub, w01 = ua * b, w11 = a * b;
            n00.add(w00 * f); d00.add(w00);
            n10.add(w10 * f); d10.add(w10);
            n01.add(w01 * f); d01.add(w01);
            n11.add(w11 * f); d11.add(w11);
        }
        wave_sync_lds();

        // corner partials of the left neighbour run (lane - 1)
        const T n10l = __shfl_up(n10.value(), 1, kWave);
        const T d10l = __shfl_up(d10.value(), 1, kWave);
        const T n11l = __shfl_up(n11.value(), 1, kWave);
        const T d11l = __shfl_up(d11.value(), 1, kWave);

        if (jd >= j_begin && tgt_ok) {
            Acc N = upN, D = upD;
            N.add(n00.value());
            N.add(n10l);
            D.add(d00.value());
            D.add(d10l);
            const T Nv = N.value(), Dv = D.value();
            const T fv = Dv > T(0) ? Nv / Dv : T(0);
            const size_t gi = (size_t)jd * nx + col;
            fgrid[gi] = fv;
            if (Dgrid) Dgrid[gi] = Dv;
            rp += (double)fv;
        }
        upN.zero();
        upD.zero();
        upN.add(n01.value());
        upN.add(n11l);
        upD.add(d01.value());
        upD.add(d11l);
    }
    if (tgt_ok) rho_part[(size_t)chunk * nx + col] = rp;
}

hipError_t launch_recon(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid,
                        double* rho_part, hipStream_t st)
{
    const int tasks = g.nstrip * g.nchunk;
    const int blocks = (tasks + kReconWaves - 1) / kReconWaves;
    const size_t esz = g.prec ? sizeof(float) : sizeof(double);
    const size_t smem = (size_t)kReconWaves * 3 * g.cap * esz;
    if (g.vdim != 1) return hipErrorNotSupported;
    static int granted[2] = {0, 0};
    {
        const void* fn = g.prec == 0 ? (const void*)k_recon_1v<0> : (const void*)k_recon_1v<1>;
        hipError_t e = ensure_lds(fn, smem, granted[g.prec]);
        if (e != hipSuccess) return e;
    }
    if (g.prec == 0)
        hipLaunchKernelGGL(k_recon_1v<0>, dim3(blocks), dim3(kWave * kReconWaves), smem, st, g,
                           *reinterpret_cast<M64*>(m), offsets, (double*)fgrid, (double*)Dgrid, rho_part);
    else
        hipLaunchKernelGGL(k_recon_1v<1>, dim3(blocks), dim3(kWave * kReconWaves), smem, st, g,
                           *reinterpret_cast<M32*>(m), offsets, (float*)fgrid, (float*)Dgrid, rho_part);
    return hipGetLastError();
}

}  // namespace avl
