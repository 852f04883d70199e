// 1D-3V weight-normalised reconstruction, Eq. (reconstruction) with the
// cloud-in-cell volume weights of Sec. 2 (a cloud of one cell volume in
// x, vx, vy, vz, so 16 grid cells share each marker).
//
// The weight of a marker for target cell (i, jx, jy, jz) factorises into an
// (x, vx) part -- the 1D-1V corner weights -- and a (vy, vz) part
// w = (1-by or by)(1-bz or bz).  A target (vy, vz) plane therefore receives
// from four dual planes (jy-cy, jz-cz), cy, cz in {0, 1}, each contributing a
// 1D-1V-like (x, vx) reconstruction with per-marker weight w.
//
// One wave owns a strip of 63 target x columns, all vx rows, and a 2x2 block
// of target (vy, vz) planes; the block draws on a 3x3 block of dual planes.
// For every dual vx row the wave walks the nine dual-plane row segments; each
// is loaded from memory once into registers (the next segment's loads go out
// once the last staging of the current one has read them) and serves every
// target plane of the block it reaches (one, two or four): per (segment,
// target) pass it is staged through LDS with that target's w, and one lane
// per run sums eight moments of (a, bx)
// weighted by f w and by w (product-sums as fused multiply-adds).  The
// corners of the runs go to the target rows jd (lower) and jd + 1 (upper, kept
// until the next dual row).  Sums are FP64: a run's sums are independent of
// the order of its markers (FixGrid in avl_device.h) and everything above
// them is added in a fixed order, with no atomics.
//
// A dual plane is still read by up to four blocks, 2.25 times on average
// instead of four times with one target plane per wave; tasks are dealt so
// that each XCD takes consecutive blocks (vy fastest), which keeps most of
// these re-reads in its L2 or in the memory-side cache.
#include "avl_device.h"

namespace avl {

template <int PREC> struct R3;
// KU: markers per lane held in registers (a segment of up to 64 KU markers is
// staged); SLOTS: staged markers in LDS, main range and wrapped run together;
// WAVES: waves per SIMD the register budget is fitted to.
template <> struct R3<0> {
    using M = M64;
    using T = double;
    static constexpr int KU = 6, SLOTS = KU * kWave + kWave, WAVES = 2;
};
template <> struct R3<1> {
    using M = M32;
    using T = float;
    static constexpr int KU = 5, SLOTS = 352, WAVES = 3;   // 11 KB of LDS
};

// One staged marker: (x, vx) offsets, and the (vy, vz) weight w and f w.
struct St3 {
    double a, b, w, fw;
};

// The (vy, vz) corner of a pass as w = (sy by + oy)(sz bz + oz): (s, o) is
// (1, 0) for the upper neighbour (weight b) and (-1, 1) for the lower (1 - b);
// either form is exact, so w is the product of the two factors as written.
struct Wsel {
    double sy, oy, sz, oz;
    __device__ Wsel(int cy, int cz)
        : sy(cy ? 1.0 : -1.0), oy(cy ? 0.0 : 1.0), sz(cz ? 1.0 : -1.0), oz(cz ? 0.0 : 1.0) {}
    __device__ double w(double by, double bz) const { return __fma_rn(sy, by, oy) * __fma_rn(sz, bz, oz); }
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
    __device__ St3 stage(const Geo& g, const Wsel& ws) const {
        int ix, jp[3];
        double a, b[3];
        double vv[3] = {vx, vy, vz};
        locate64<3>(g, x, vv, ix, jp, a, b);
        St3 s;
        s.a = a;
        s.b = b[0];
        s.w = ws.w(b[1], b[2]);
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
    __device__ St3 stage(const Geo&, const Wsel& ws) const {
        St3 s;
        s.a = a;
        s.b = bx;
        s.w = ws.w(by, bz);
        s.fw = (double)f * s.w;
        return s;
    }
};

// Lane l receives lane l-1's value (lane 0 receives 0): a DPP shift of the
// whole wavefront by one lane, two 32-bit moves for a double.
__device__ __forceinline__ double from_left3(double v)
{
    constexpr int kWaveShr1 = 0x138;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kWaveShr1, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kWaveShr1, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void wave_sync_lds3()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct Seg3 {
    int lo, nmain, wbeg, wlen;
};

template <int PREC>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(R3<PREC>::WAVES)))
void k_recon_3v(Geo g, typename R3<PREC>::M m, const int* __restrict__ offsets, typename R3<PREC>::T* __restrict__ fgrid,
                typename R3<PREC>::T* __restrict__ Dgrid, double* __restrict__ rho_part, int tasks_per_xcd)
{
    using T = typename R3<PREC>::T;
    constexpr int KU = R3<PREC>::KU, CAP = KU * kWave, SLOTS = R3<PREC>::SLOTS;
    __shared__ St3 st[SLOTS];
    const int lane = threadIdx.x;
    const int nby = (g.nv[1] + 1) >> 1, nbz = (g.nv[2] + 1) >> 1;
    const int ntask = g.nstrip * nby * nbz;
    const int task = (blockIdx.x & 7) * tasks_per_xcd + (blockIdx.x >> 3);
    if ((blockIdx.x >> 3) >= tasks_per_xcd || task >= ntask) return;
    // task = (strip * nbz + bz) * nby + by: consecutive tasks are neighbouring blocks
    const int by = task % nby;
    const int bz = (task / nby) % nbz;
    const int strip = task / (nby * nbz);
    // target planes (jy0 + ty, jz0 + tz), ty < nyt, tz < nzt; dual planes
    // (jy0 - 1 + iy, jz0 - 1 + iz), iy < ndy = nyt + 1, iz < ndz = nzt + 1
    const int jy0 = 2 * by, jz0 = 2 * bz;
    const int nyt = min(2, g.nv[1] - jy0), nzt = min(2, g.nv[2] - jz0);
    const int ndy = nyt + 1, ndz = nzt + 1;
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

    // Segments are visited row by row (dual vx row r = jd + 1 in [0, nvx]),
    // and within a row plane by plane (iy fastest).  A cursor names a
    // segment; run bounds are fetched two segments ahead, markers one.
    struct Cur {
        int r, iy, iz;
    };
    auto advance = [&](Cur& c) {
        if (++c.iy == ndy) {
            c.iy = 0;
            if (++c.iz == ndz) {
                c.iz = 0;
                ++c.r;
            }
        }
    };
    auto seg_bounds = [&](const Cur& c, int& beg, int& end) {
        beg = 0;
        end = 0;
        if (c.r <= nvx && run_ok) {
            const int row = ((jz0 + c.iz) * rowsy + (jy0 + c.iy)) * rowsx + c.r;
            const int bk = row * nx + colw;
            beg = offsets[bk];
            end = offsets[bk + 1];
        }
    };
    auto make = [&](int beg, int end) {
        Seg3 s;
        s.lo = __builtin_amdgcn_readlane(beg, first_lane);
        const int hi = __builtin_amdgcn_readlane(end, last_lane);
        s.wbeg = __builtin_amdgcn_readlane(beg, 0);
        const int wend = __builtin_amdgcn_readlane(end, 0);
        s.nmain = hi - s.lo;
        s.wlen = wrapped ? wend - s.wbeg : 0;
        return s;
    };
    auto fits = [&](const Seg3& s) { return s.nmain <= CAP && s.wlen <= kWave && s.nmain + s.wlen <= SLOTS; };

    Raw3<PREC> regs[KU], wreg;
    auto prefetch = [&](const Seg3& s) {
        if (!fits(s)) return;
#pragma unroll
        for (int k = 0; k < KU; ++k) {
            const int p = lane + k * kWave;
            if (p < s.nmain) regs[k].load(m, g, s.lo + p);
        }
        if (lane < s.wlen) wreg.load(m, g, s.wbeg + lane);
    };

    Cur cur{0, 0, 0}, ahead{0, 0, 0};
    int beg, end, nbeg, nend;
    seg_bounds(ahead, beg, end);
    Seg3 seg = make(beg, end);
    prefetch(seg);
    advance(ahead);
    seg_bounds(ahead, nbeg, nend);
    advance(ahead);

    // per target plane t = tz * 2 + ty: row jd so far (cN) and row jd + 1 (uN)
    double cN[4] = {0.0, 0.0, 0.0, 0.0}, cD[4] = {0.0, 0.0, 0.0, 0.0};
    double uN[4] = {0.0, 0.0, 0.0, 0.0}, uD[4] = {0.0, 0.0, 0.0, 0.0};
    double rp[4] = {0.0, 0.0, 0.0, 0.0};

    while (cur.r <= nvx) {
        // issue priority from progress (the FP32 form; the FP64 form's three
        // waves a compute unit ran slower with it)
        if constexpr (PREC == 1) prio_by_progress(cur.r, nvx + 1);
        const int iy = cur.iy, iz = cur.iz;
        const bool staged = fits(seg);
        const int p0 = staged ? ((wrapped && lane == 0) ? seg.nmain : beg - seg.lo) : beg;
        const int len = end - beg;
        const Seg3 nxt = make(nbeg, nend);
        // the last target plane this dual plane reaches; the next segment's
        // loads go out once its staging no longer needs the registers
        const int tlast = min(iz, nzt - 1) * 2 + min(iy, nyt - 1);

#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ty = t & 1, tz = t >> 1;
            const int cy = ty - iy + 1, cz = tz - iz + 1;     // corner of the dual plane
            if (ty >= nyt || tz >= nzt || cy < 0 || cy > 1 || cz < 0 || cz > 1) continue;
            const Wsel ws(cy, cz);
            if (staged) {
#pragma unroll
                for (int k = 0; k < KU; ++k) {
                    if (k * kWave >= seg.nmain) break;         // wave-uniform
                    const int q = lane + k * kWave;
                    if (q < seg.nmain) st[q] = regs[k].stage(g, ws);
                }
                if (lane < seg.wlen) st[seg.nmain + lane] = wreg.stage(g, ws);
            }
            if (t == tlast) prefetch(nxt);
            wave_sync_lds3();
            // moments of (a, b) weighted by w and by f w, order-independent
            // (FixGrid in avl_device.h): the w sums on a grid fitted to the
            // run's largest w, the f w sums on one fitted to its largest |f w|.
            // For f = c = 2^k on every marker every f w is c w exactly, the two
            // grids differ by exactly c, and f = c comes out exactly
            unsigned kw = 0, kf = 0;
            if (staged) {
                for (int k = 0; k < len; ++k) {
                    kw = max(kw, fix_key(st[p0 + k].w));
                    kf = max(kf, fix_key(st[p0 + k].fw));
                }
            } else {
                for (int k = 0; k < len; ++k) {
                    Raw3<PREC> rr;
                    rr.load(m, g, p0 + k);
                    const St3 e = rr.stage(g, ws);
                    kw = max(kw, fix_key(e.w));
                    kf = max(kf, fix_key(e.fw));
                }
            }
            const int ew = len > 0 ? fix_exp_of_key(kw, 0.0) : -1100;
            const int ef = len > 0 ? fix_exp_of_key(kf, 0.0) : -1100;
            const double Cw = fix_origin(ew, len), Cf = fix_origin(ef, len);
            double Sw = Cw, Saw = Cw, Sbw = Cw, Sabw = Cw;
            double Sf = Cf, Saf = Cf, Sbf = Cf, Sabf = Cf;
            auto pin8 = [&]() {
                fixsum_pin(Sw); fixsum_pin(Saw); fixsum_pin(Sbw); fixsum_pin(Sabw);
                fixsum_pin(Sf); fixsum_pin(Saf); fixsum_pin(Sbf); fixsum_pin(Sabf);
            };
            if (staged) {
                // FP64 rounding toward -infinity: each operation adds floor(term / q) q
                fixsum_round_down();
                pin8();
#pragma unroll 2
                for (int k = 0; k < len; ++k) {
                    const St3 e = st[p0 + k];
                    const double ab = e.a * e.b;
                    Sw += e.w;
                    Saw = fma(e.a, e.w, Saw);
                    Sbw = fma(e.b, e.w, Sbw);
                    Sabw = fma(ab, e.w, Sabw);
                    Sf += e.fw;
                    Saf = fma(e.a, e.fw, Saf);
                    Sbf = fma(e.b, e.fw, Sbf);
                    Sabf = fma(ab, e.fw, Sabf);
                }
                pin8();
                fixsum_round_nearest();
                pin8();
            } else {
                // staged per marker in the default rounding (the FP64 form
                // locates it here), then added in the rounding toward -infinity
                for (int k = 0; k < len; ++k) {
                    Raw3<PREC> rr;
                    rr.load(m, g, p0 + k);
                    St3 e = rr.stage(g, ws);
                    fixsum_pin(e.a); fixsum_pin(e.b); fixsum_pin(e.w); fixsum_pin(e.fw);
                    fixsum_round_down();
                    pin8();
                    const double ab = e.a * e.b;
                    Sw += e.w;
                    Saw = fma(e.a, e.w, Saw);
                    Sbw = fma(e.b, e.w, Sbw);
                    Sabw = fma(ab, e.w, Sabw);
                    Sf += e.fw;
                    Saf = fma(e.a, e.fw, Saf);
                    Sbf = fma(e.b, e.fw, Sbf);
                    Sabf = fma(ab, e.fw, Sabf);
                    pin8();
                    fixsum_round_nearest();
                    pin8();
                }
            }
            wave_sync_lds3();
            Sw -= Cw; Saw -= Cw; Sbw -= Cw; Sabw -= Cw;
            Sf -= Cf; Saf -= Cf; Sbf -= Cf; Sabf -= Cf;
            const double n11 = Sabf, n10 = Saf - Sabf, n01 = Sbf - Sabf, n00 = (Sf - Saf) - n01;
            const double d11 = Sabw, d10 = Saw - Sabw, d01 = Sbw - Sabw, d00 = (Sw - Saw) - d01;
            cN[t] += n00 + from_left3(n10);
            cD[t] += d00 + from_left3(d10);
            uN[t] += n01 + from_left3(n11);
            uD[t] += d01 + from_left3(d11);
        }

        if (iy == ndy - 1 && iz == ndz - 1) {
            // target row jd = r - 1 of every plane of the block is complete
            const int jd = cur.r - 1;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int ty = t & 1, tz = t >> 1;
                if (ty < nyt && tz < nzt && jd >= 0 && tgt_ok) {
                    const double fv = cD[t] > 0.0 ? cN[t] / cD[t] : 0.0;
                    const size_t gi = (((size_t)(jz0 + tz) * g.nv[1] + (jy0 + ty)) * nvx + jd) * nx + col;
                    fgrid[gi] = (T)fv;
                    if (Dgrid) Dgrid[gi] = (T)cD[t];
                    rp[t] += (double)(T)fv;
                }
                cN[t] = uN[t];
                cD[t] = uD[t];
                uN[t] = 0.0;
                uD[t] = 0.0;
            }
        }

        advance(cur);
        beg = nbeg;
        end = nend;
        seg = nxt;
        seg_bounds(ahead, nbeg, nend);
        advance(ahead);
    }
    if constexpr (PREC == 1) __builtin_amdgcn_s_setprio(0);
    if (tgt_ok) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ty = t & 1, tz = t >> 1;
            if (ty < nyt && tz < nzt) rho_part[((size_t)(jz0 + tz) * g.nv[1] + (jy0 + ty)) * nx + col] = rp[t];
        }
    }
}

size_t recon3_scratch_bytes(const Geo&) { return 0; }

hipError_t launch_recon3(const Geo& g, void* m, const int* offsets, void* fgrid, void* Dgrid, double* rho_part,
                         void*, hipStream_t st)
{
    const int tasks = g.nstrip * ((g.nv[1] + 1) / 2) * ((g.nv[2] + 1) / 2);
    const int per_xcd = (tasks + 7) / 8;
    const int blocks = per_xcd * 8;
    if (g.prec == 0)
        launch(k_recon_3v<0>, dim3(blocks), dim3(kWave), 0, st, g, *reinterpret_cast<M64*>(m), offsets,
                           (double*)fgrid, (double*)Dgrid, rho_part, per_xcd);
    else
        launch(k_recon_3v<1>, dim3(blocks), dim3(kWave), 0, st, g, *reinterpret_cast<M32*>(m), offsets,
                           (float*)fgrid, (float*)Dgrid, rho_part, per_xcd);
    return hipGetLastError();
}

}  // namespace avl
