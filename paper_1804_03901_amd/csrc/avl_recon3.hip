// 1D-3V weight-normalised reconstruction, Eq. (reconstruction) with the
// cloud-in-cell volume weights of Sec. 2 (a cloud of one cell volume in
// x, vx, vy, vz, so 16 grid cells share each marker).
//
// The weight of a marker for target cell (i, jx, jy, jz) factorises into an
// (x, vx) part -- the 1D-1V corner weights -- and a (vy, vz) part
// w = (1-by or by)(1-bz or bz).  A target (vy, vz) plane therefore receives
// from four dual planes (jy-cy, jz-cz), cy, cz in {0, 1}, each contributing a
// 1D-1V-like (x, vx) reconstruction with per-marker weight w.  One wave owns
// a strip of 63 target x columns and all vx rows of one target plane; for
// every vx row it walks the four dual planes in a fixed order, staging each
// row segment through LDS (the next segment is prefetched into registers while
// the current one is summed), and sums per run eight moments of (a, bx)
// weighted by f w and by w (product-sums as fused multiply-adds).  Sums are
// FP64 and in a fixed order: no atomics.
//
// Neighbouring target planes read the same dual planes; tasks are dealt so
// that each XCD takes consecutive target planes (vy fastest), which keeps the
// re-reads in its L2 or in the memory-side cache.
#include "avl_device.h"

namespace avl {

constexpr int kKU3 = 8;                       // prefetched markers per lane (segment up to 512)
constexpr int kCap3 = kWave * kKU3;

template <int PREC> struct R3;
template <> struct R3<0> {
    using M = M64;
    using T = double;
};
template <> struct R3<1> {
    using M = M32;
    using T = float;
};

// One staged marker: (x, vx) offsets, and the (vy, vz) weight w and f w.
struct St3 {
    double a, b, w, fw;
};

// Raw marker fields as loaded.
template <int PREC> struct Raw3;
template <> struct Raw3<0> {
    double x, vx, vy, vz, f;
    __device__ void load(const M64& m, const Geo& g, int q) {
        x = m.x[q];
        vx = m.v[q];
        vy = m.v[(size_t)g.np + q];
        vz = m.v[2 * (size_t)g.np + q];
        f = m.f[q];
    }
    __device__ St3 stage(const Geo& g, int cy, int cz) const {
        int ix, jp[3];
        double a, b[3];
        double vv[3] = {vx, vy, vz};
        locate64<3>(g, x, vv, ix, jp, a, b);
        St3 s;
        s.a = a;
        s.b = b[0];
        s.w = (cy ? b[1] : 1.0 - b[1]) * (cz ? b[2] : 1.0 - b[2]);
        s.fw = f * s.w;
        return s;
    }
};
template <> struct Raw3<1> {
    float a, bx, by, bz, f;
    __device__ void load(const M32& m, const Geo& g, int q) {
        a = m.a[q];
        bx = m.b[q];
        by = m.b[(size_t)g.np + q];
        bz = m.b[2 * (size_t)g.np + q];
        f = m.f[q];
    }
    __device__ St3 stage(const Geo&, int cy, int cz) const {
        const double y = by, zz = bz;
        St3 s;
        s.a = a;
        s.b = bx;
        s.w = (cy ? y : 1.0 - y) * (cz ? zz : 1.0 - zz);
        s.fw = (double)f * s.w;
        return s;
    }
};

__device__ __forceinline__ void wave_sync_lds3()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct Seg3 {
    int lo, nmain, wbeg, wlen;
};

template <int PREC>
__global__ __launch_bounds__(kWave) void k_recon_3v(Geo g, typename R3<PREC>::M m, const int* __restrict__ offsets,
                                                    typename R3<PREC>::T* __restrict__ fgrid,
                                                    typename R3<PREC>::T* __restrict__ Dgrid,
                                                    double* __restrict__ rho_part, int tasks_per_xcd)
{
    using T = typename R3<PREC>::T;
    __shared__ St3 st[kCap3 + kWave];
    const int lane = threadIdx.x;
    const int ntask = g.nstrip * g.nv[1] * g.nv[2];
    const int task = (blockIdx.x & 7) * tasks_per_xcd + (blockIdx.x >> 3);
    if ((blockIdx.x >> 3) >= tasks_per_xcd || task >= ntask) return;
    // task = (strip * nvz + jz) * nvy + jy: consecutive tasks are neighbouring planes
    const int jy = task % g.nv[1];
    const int jz = (task / g.nv[1]) % g.nv[2];
    const int strip = task / (g.nv[1] * g.nv[2]);
    const int nx = g.nx, nvx = g.nv[0];
    const int col = strip * kReconCols - 1 + lane;
    const bool run_ok = col < nx;
    const int colw = col < 0 ? nx - 1 : col;
    const bool tgt_ok = lane >= 1 && col < nx;
    const bool wrapped = (strip == 0);
    const int first_lane = wrapped ? 1 : 0;
    const int last_col = min(strip * kReconCols + kReconCols - 1, nx - 1);
    const int last_lane = last_col - (strip * kReconCols - 1);
    const int rowsy = g.nv[1] + 1, rowsx = nvx + 1;

    // segment s = (dual x-velocity row jd in [-1, nvx-1]) * 4 + (vy, vz) corner p;
    // p = cz * 2 + cy names the dual plane (jy - cy, jz - cz)
    const int nseg = (nvx + 1) * 4;
    auto seg_bounds = [&](int s, int& beg, int& end) {
        beg = 0;
        end = 0;
        if (s < nseg && run_ok) {
            const int jd = s / 4 - 1, p = s & 3;
            const int jyd = jy - (p & 1), jzd = jz - (p >> 1);
            const int row = ((jzd + 1) * rowsy + (jyd + 1)) * rowsx + (jd + 1);
            const int bk = row * nx + colw;
            beg = offsets[bk];
            end = offsets[bk + 1];
        }
    };
    auto make = [&](int beg, int end) {
        Seg3 s;
        s.lo = __shfl(beg, first_lane, kWave);
        const int hi = __shfl(end, last_lane, kWave);
        s.wbeg = __shfl(beg, 0, kWave);
        const int wend = __shfl(end, 0, kWave);
        s.nmain = hi - s.lo;
        s.wlen = wrapped ? wend - s.wbeg : 0;
        return s;
    };
    auto fits = [&](const Seg3& s) { return s.nmain <= kCap3 && s.wlen <= kWave; };

    Raw3<PREC> regs[kKU3], wreg;
    auto prefetch = [&](const Seg3& s) {
        if (!fits(s)) return;
#pragma unroll
        for (int k = 0; k < kKU3; ++k) {
            const int p = lane + k * kWave;
            if (p < s.nmain) regs[k].load(m, g, s.lo + p);
        }
        if (lane < s.wlen) wreg.load(m, g, s.wbeg + lane);
    };

    int beg, end, nbeg, nend;
    seg_bounds(0, beg, end);
    Seg3 seg = make(beg, end);
    prefetch(seg);
    seg_bounds(1, nbeg, nend);

    double upN[4] = {0.0, 0.0, 0.0, 0.0}, upD[4] = {0.0, 0.0, 0.0, 0.0};
    double rowN = 0.0, rowD = 0.0;
    double rp = 0.0;

    for (int s = 0; s < nseg; ++s) {
        const int jd = s / 4 - 1, p = s & 3;
        const int cy = p & 1, cz = p >> 1;
        const bool staged = fits(seg);
        if (staged) {
#pragma unroll
            for (int k = 0; k < kKU3; ++k) {
                const int q = lane + k * kWave;
                if (q < seg.nmain) st[q] = regs[k].stage(g, cy, cz);
            }
            if (lane < seg.wlen) st[seg.nmain + lane] = wreg.stage(g, cy, cz);
        }
        wave_sync_lds3();
        const int p0 = staged ? ((wrapped && lane == 0) ? seg.nmain : beg - seg.lo) : beg;
        const int len = end - beg;
        Seg3 nseg_ = make(nbeg, nend);
        if (s + 1 < nseg) prefetch(nseg_);
        int nnbeg, nnend;
        seg_bounds(s + 2, nnbeg, nnend);

        // moments of (a, b) weighted by w and by f w
        double Sw = 0, Saw = 0, Sbw = 0, Sabw = 0, Sf = 0, Saf = 0, Sbf = 0, Sabf = 0;
        if (staged) {
            for (int k = 0; k < len; ++k) {
                const St3 e = st[p0 + k];
                const double ab = e.a * e.b;
                Sw += e.w;
                Saw = __fma_rn(e.a, e.w, Saw);
                Sbw = __fma_rn(e.b, e.w, Sbw);
                Sabw = __fma_rn(ab, e.w, Sabw);
                Sf += e.fw;
                Saf = __fma_rn(e.a, e.fw, Saf);
                Sbf = __fma_rn(e.b, e.fw, Sbf);
                Sabf = __fma_rn(ab, e.fw, Sabf);
            }
        } else {
            for (int k = 0; k < len; ++k) {
                Raw3<PREC> r;
                r.load(m, g, p0 + k);
                const St3 e = r.stage(g, cy, cz);
                const double ab = e.a * e.b;
                Sw += e.w;
                Saw = __fma_rn(e.a, e.w, Saw);
                Sbw = __fma_rn(e.b, e.w, Sbw);
                Sabw = __fma_rn(ab, e.w, Sabw);
                Sf += e.fw;
                Saf = __fma_rn(e.a, e.fw, Saf);
                Sbf = __fma_rn(e.b, e.fw, Sbf);
                Sabf = __fma_rn(ab, e.fw, Sabf);
            }
        }
        wave_sync_lds3();
        const double n11 = Sabf, n10 = Saf - Sabf, n01 = Sbf - Sabf, n00 = (Sf - Saf) - n01;
        const double d11 = Sabw, d10 = Saw - Sabw, d01 = Sbw - Sabw, d00 = (Sw - Saw) - d01;
        const double n10l = __shfl_up(n10, 1, kWave);
        const double d10l = __shfl_up(d10, 1, kWave);
        const double n11l = __shfl_up(n11, 1, kWave);
        const double d11l = __shfl_up(d11, 1, kWave);

        // target row jd of this plane: the carry from dual row jd-1 plus this row
        double cN = 0.0, cD = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q == p) {
                cN = upN[q];
                cD = upD[q];
                upN[q] = n01 + n11l;
                upD[q] = d01 + d11l;
            }
        rowN += (cN + n00) + n10l;
        rowD += (cD + d00) + d10l;
        if (p == 3) {
            if (jd >= 0 && tgt_ok) {
                const double fv = rowD > 0.0 ? rowN / rowD : 0.0;
                const size_t gi = (((size_t)jz * g.nv[1] + jy) * nvx + jd) * nx + col;
                fgrid[gi] = (T)fv;
                if (Dgrid) Dgrid[gi] = (T)rowD;
                rp += (double)(T)fv;
            }
            rowN = 0.0;
            rowD = 0.0;
        }

        beg = nbeg;
        end = nend;
        nbeg = nnbeg;
        nend = nnend;
        seg = nseg_;
    }
    if (tgt_ok) rho_part[((size_t)jz * g.nv[1] + jy) * nx + col] = rp;
}

size_t recon3_scratch_bytes(const Geo&) { return 0; }

hipError_t launch_recon3(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid, double* rho_part,
                         void*, hipStream_t st)
{
    const int tasks = g.nstrip * g.nv[1] * g.nv[2];
    const int per_xcd = (tasks + 7) / 8;
    const int blocks = per_xcd * 8;
    if (g.prec == 0)
        hipLaunchKernelGGL(k_recon_3v<0>, dim3(blocks), dim3(kWave), 0, st, g, *reinterpret_cast<M64*>(m), offsets,
                           (double*)fgrid, (double*)Dgrid, rho_part, per_xcd);
    else
        hipLaunchKernelGGL(k_recon_3v<1>, dim3(blocks), dim3(kWave), 0, st, g, *reinterpret_cast<M32*>(m), offsets,
                           (float*)fgrid, (float*)Dgrid, rho_part, per_xcd);
    return hipGetLastError();
}

}  // namespace avl
