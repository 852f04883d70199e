// Charge density, spectral field solve and per-step diagnostics in one launch.
//
// rho_i = q * prod(dv) * sum_j f_ij is assembled from the reconstruction's
// per-chunk column partials (Sec. 2: the moment is a plain sum over velocity
// cells at fixed x).  The field follows Eq. (poissonk) with the softening of
// Eq. (kappasoftening): a forward FFT of rho, multiplication by
// -i c_p kappa_m / K_m^2 (a host-built table that is zero at m = 0 and at the
// Nyquist mode), and an inverse FFT, taken as the forward transform of the
// conjugate spectrum (E is real, so E = Re FFT(conj(E_hat)) / nx).  The FFT is
// a self-sorting (Stockham) radix-4 transform in LDS, with one radix-2 stage
// first when log2(nx) is odd; each stage reads all its inputs, synchronises,
// then writes, so one nx-point buffer suffices.  FP64 throughout.
// Also here: marker validation/conversion kernels and the copy probe.
#include <algorithm>

#include "avl_device.h"

namespace avl {

static int g_lds_limit = 65536;
void set_lds_limit(int bytes) { g_lds_limit = bytes; }
int lds_limit() { return g_lds_limit; }

constexpr int kFT = kFieldThreads;            // threads of a field block
constexpr int kFieldGroups = kFT / 64;         // chunk groups per 64-column block

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// e^{-2 pi i idx / N} for idx in [0, N) from the half table (idx < N/2),
// using w^(idx + N/2) = -w^idx; no branch, one LDS read.
__device__ __forceinline__ double2 twiddle(const double2* stw, int idx, int half_n)
{
    const double2 t = stw[idx & (half_n - 1)];
    const double s = (idx & half_n) ? -1.0 : 1.0;
    return make_double2(s * t.x, s * t.y);
}

// One Stockham stage of radix R (2 or 4) for the current span Ns: butterfly j
// takes inputs j + r*N/R, twiddled by w^(r*(j mod Ns)*N/(Ns*R)), and writes
// output r to (j - j mod Ns)*R + j mod Ns + r*Ns.
template <int R>
__device__ __forceinline__ void stockham_stage(double2* z, const double2* stw, int lgN, int lgNs)
{
    constexpr int lgR = R == 2 ? 1 : 2;
    constexpr int MAXJ = (kMaxNx / R + kFT - 1) / kFT;
    const int N = 1 << lgN, nb = N >> lgR, half_n = N >> 1;
    const int Ns = 1 << lgNs, tshift = lgN - lgNs - lgR;
    double2 v[MAXJ][R];
    int dst[MAXJ];
#pragma unroll
    for (int q = 0; q < MAXJ; ++q) {
        const int j = threadIdx.x + q * kFT;
        dst[q] = -1;
        if (j < nb) {
            const int k = j & (Ns - 1);
            const int t = k << tshift;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 x = z[j + r * nb];
                v[q][r] = r == 0 ? x : cmul(x, twiddle(stw, r * t, half_n));
            }
            if (R == 2) {
                const double2 a = v[q][0], b = v[q][1];
                v[q][0] = make_double2(a.x + b.x, a.y + b.y);
                v[q][1] = make_double2(a.x - b.x, a.y - b.y);
            } else {
                const double2 a = make_double2(v[q][0].x + v[q][2].x, v[q][0].y + v[q][2].y);
                const double2 b = make_double2(v[q][0].x - v[q][2].x, v[q][0].y - v[q][2].y);
                const double2 c = make_double2(v[q][1].x + v[q][3].x, v[q][1].y + v[q][3].y);
                const double2 d = make_double2(v[q][1].x - v[q][3].x, v[q][1].y - v[q][3].y);
                v[q][0] = make_double2(a.x + c.x, a.y + c.y);
                v[q][1] = make_double2(b.x + d.y, b.y - d.x);      // b - i d
                v[q][2] = make_double2(a.x - c.x, a.y - c.y);
                v[q][3] = make_double2(b.x - d.y, b.y + d.x);      // b + i d
            }
            dst[q] = (j - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXJ; ++q)
        if (dst[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) z[dst[q] + r * Ns] = v[q][r];
        }
    __syncthreads();
}

// In-place forward DFT, X_m = sum_n z_n e^{-2 pi i m n / N}, natural order in and out.
__device__ void fft_forward(double2* z, const double2* stw, int lgN)
{
    int lgNs = 0;
    if (lgN & 1) {
        stockham_stage<2>(z, stw, lgN, 0);
        lgNs = 1;
    }
    for (; lgNs < lgN; lgNs += 2) stockham_stage<4>(z, stw, lgN, lgNs);
}


// Charge density, part 1: block (column group, slice) sums the chunk partials
// of its slice for 64 x cells (16 groups of chunks per column, combined in a
// fixed order) into rho_slices[slice][i].
__device__ __forceinline__ void rho_block(const Geo& g, const double* __restrict__ rho_part,
                                          double* __restrict__ rho_slices, int nslice, int blk)
{
    __shared__ double colsum[kFT];
    const int nx = g.nx, tid = threadIdx.x;
    const int ncg = (nx + 63) >> 6;
    const int cg = blk % ncg, sl = blk / ncg;
    const int c = tid & 63, grp = tid >> 6;
    const int i = cg * 64 + c;
    const int per = (g.nchunk + nslice - 1) / nslice;
    const int ch_lo = sl * per, ch_hi = min(g.nchunk, ch_lo + per);
    double acc = 0.0;
    if (i < nx) {
        // batches of 16 independent loads (chunks grp, grp+16, ...), summed in order
        for (int ch0 = ch_lo + grp; ch0 < ch_hi; ch0 += 16 * kFieldGroups) {
            double v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int ch = ch0 + kFieldGroups * k;
                v[k] = ch < ch_hi ? rho_part[(size_t)ch * nx + i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += v[k];
        }
    }
    colsum[grp * 64 + c] = acc;
    __syncthreads();
    if (grp == 0 && i < nx) {
        double t = 0.0;
        for (int k = 0; k < kFieldGroups; ++k) t += colsum[k * 64 + c];
        rho_slices[(size_t)sl * nx + i] = t;
    }
}

__global__ __launch_bounds__(kFT) void k_rho(Geo g, const double* __restrict__ rho_part,
                                             double* __restrict__ rho_slices, int nslice)
{
    rho_block(g, rho_part, rho_slices, nslice, blockIdx.x);
}

// Charge density, part 2, and the field solve, one block: rho_i = q prod(dv)
// * (sum of the slices in order) or the caller's rho, then the spectral solve
// and the diagnostics.  Every global read the block needs is issued up front
// so that their latencies overlap.
__device__ __forceinline__ void solve_block(const Geo& g, const double* __restrict__ rho_slices, int nslice,
                                            const double* __restrict__ rho_in, double* __restrict__ rho,
                                            double* __restrict__ E_out, const double2* __restrict__ tw,
                                            const double* __restrict__ green, double* __restrict__ diag_ring,
                                            long long* __restrict__ step_ctr, int write_diag,
                                            double* __restrict__ W_out, int* __restrict__ flags)
{
    constexpr int Q = kMaxNx / kFT;               // grid points per thread at most
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, lg = g.lognx;
    const int half_n = nx >> 1;
    double2* z = reinterpret_cast<double2*>(smem);
    double2* stw = z + nx;
    const int tid = threadIdx.x;

    const long long ctr = (write_diag && tid == 0) ? *step_ctr : 0;
    double rv[Q], gv[Q];
    double2 twv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = tid + q * kFT;
        rv[q] = 0.0;
        gv[q] = 0.0;
        twv[q] = make_double2(0.0, 0.0);
        if (i < nx) {
            if (rho_in) {
                rv[q] = rho_in[i];
            } else {
                for (int s = 0; s < nslice; ++s) rv[q] += rho_slices[(size_t)s * nx + i];
            }
            gv[q] = green[i];
            if (i < half_n) twv[q] = tw[i];
        }
    }
    // The k = 0 mode is dropped (E_hat_0 = 0), so the mean of rho cannot
    // change E; it is subtracted before the transform so that a large mean
    // (the neutralised charge) does not leak into the other modes through the
    // rounding of the butterflies.  The mean is a fixed-order block sum.
    __shared__ double s_sum[kFT / kWave];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = tid + q * kFT;
        if (i < nx) {
            if (!rho_in) {
                rv[q] *= g.q_vol;
                rho[i] = rv[q];
            }
            part += rv[q];
            if (i < half_n) stw[i] = twv[q];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    if ((tid & (kWave - 1)) == 0) s_sum[tid / kWave] = part;
    __syncthreads();
    double total = 0.0;
    for (int w = 0; w < kFT / kWave; ++w) total += s_sum[w];
    const double mean = total / nx;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = tid + q * kFT;
        if (i < nx) z[i] = make_double2(rv[q] - mean, 0.0);
    }
    __syncthreads();
    // rho_hat_m = sum_i rho_i exp(-2 pi i m i / nx)
    fft_forward(z, stw, lg);
    // conj(E_hat_m) with E_hat_m = -i (c_p kappa_m / K_m^2) rho_hat_m
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int m = tid + q * kFT;
        if (m < nx) {
            const double2 r = z[m];
            z[m] = make_double2(gv[q] * r.y, gv[q] * r.x);
        }
    }
    __syncthreads();
    fft_forward(z, stw, lg);
    const double inv_n = 1.0 / nx;
    int bad = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = tid + q * kFT;
        if (i < nx) {
            const double E = z[i].x * inv_n;
            E_out[i] = E;
            if (!isfinite(E)) bad = 1;
        }
    }
    if (bad) atomicOr(flags, FLAG_NONFINITE);
    if (tid >= kWave) return;
    // diagnostics by the first wave: sum E^2 and the mode-1 coefficient of E,
    // lane-strided then a shuffle tree (fixed order)
    double sw = 0.0, sre = 0.0, sim = 0.0;
    for (int i = tid; i < nx; i += kWave) {
        const double E = z[i].x * inv_n;
        const double2 w = twiddle(stw, i, half_n);
        sw += E * E;
        sre += E * w.x;
        sim += E * w.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sw += __shfl_xor(sw, o, kWave);
        sre += __shfl_xor(sre, o, kWave);
        sim += __shfl_xor(sim, o, kWave);
    }
    if (tid == 0) {
        const double W = sw * g.dx / (2.0 * g.cp);
        const double m1 = 2.0 / nx * sqrt(sre * sre + sim * sim);
        if (W_out) *W_out = W;
        if (write_diag) {
            diag_ring[2 * (ctr % kDiagCap)] = W;
            diag_ring[2 * (ctr % kDiagCap) + 1] = m1;
            *step_ctr = ctr + 1;
        }
    }
}

__global__ __launch_bounds__(kFT) void k_solve(Geo g, const double* __restrict__ rho_slices, int nslice,
                                               const double* __restrict__ rho_in, double* __restrict__ rho,
                                               double* __restrict__ E_out, const double2* __restrict__ tw,
                                               const double* __restrict__ green, double* __restrict__ diag_ring,
                                               long long* __restrict__ step_ctr, int write_diag,
                                               double* __restrict__ W_out, int* __restrict__ flags)
{
    solve_block(g, rho_slices, nslice, rho_in, rho, E_out, tw, green, diag_ring, step_ctr, write_diag, W_out, flags);
}

// Batched charge density and field solve: rho blocks of every instance in one
// launch, then one solve block per instance.
__global__ __launch_bounds__(kFT) void k_rho_b(const BInst* __restrict__ tab, const int* __restrict__ pre, int ninst)
{
    const int* pr = pre + BPRE_RHO * (ninst + 1);
    const int i = find_inst(pr, ninst, blockIdx.x);
    const BInst& I = tab[i];
    rho_block(I.g, I.rho_part, I.rho_slices, I.nslice, blockIdx.x - pr[i]);
}

__global__ __launch_bounds__(kFT) void k_solve_b(const BInst* __restrict__ tab, int write_diag)
{
    const BInst& I = tab[blockIdx.x];
    solve_block(I.g, I.rho_slices, I.nslice, nullptr, I.rho, I.E, I.tw, I.green, I.diag, I.ctr, write_diag, nullptr,
                I.flags);
}

hipError_t launch_field_batch(const BInst* tab, const int* pre, int ninst, int rho_blocks, int max_nx, int write_diag,
                              hipStream_t st)
{
    const size_t smem = (sizeof(double2) + sizeof(double2) / 2) * max_nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_solve_b, smem, granted);
    if (e != hipSuccess) return e;
    if (rho_blocks > 0) hipLaunchKernelGGL(k_rho_b, dim3(rho_blocks), dim3(kFT), 0, st, tab, pre, ninst);
    hipLaunchKernelGGL(k_solve_b, dim3(ninst), dim3(kFT), smem, st, tab, write_diag);
    return hipGetLastError();
}

// Chunk slices of the rho reduction: at most 256 chunk partials per block.
int field_slices(const Geo& g) { return std::max(1, std::min(kMaxFieldSlices, (g.nchunk + 255) / 256)); }

// ---------------------------------------------------------------------------
// Several species in one field (Sec. 2: rho is the sum over species of
// q_s times the velocity integral of f_s; one field pushes every species).
// ---------------------------------------------------------------------------

// Per column: each species' rho (its slices in slice order, or its rho when
// from_rho is set, times q prod(dv)), and the total in species order.
__global__ void k_species_rho(const Species* __restrict__ sp, int ns, int nx, int from_rho,
                              double* __restrict__ rho_total)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += gridDim.x * blockDim.x) {
        double tot = 0.0;
        for (int s = 0; s < ns; ++s) {
            double r;
            if (from_rho) {
                r = sp[s].rho[i];
            } else {
                r = 0.0;
                for (int k = 0; k < sp[s].nslice; ++k) r += sp[s].rho_slices[(size_t)k * nx + i];
                r *= sp[s].q_vol;
                sp[s].rho[i] = r;
            }
            tot += r;
        }
        rho_total[i] = tot;
    }
}

// The field solved into species 0's buffer, copied to the others.
__global__ void k_broadcast_E(const Species* __restrict__ sp, int ns, int nx)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += gridDim.x * blockDim.x) {
        const double e = sp[0].E[i];
        for (int s = 1; s < ns; ++s) sp[s].E[i] = e;
    }
}

hipError_t launch_rho_slices(const Geo& g, const double* rho_part, double* rho_slices, hipStream_t st)
{
    const int nslice = field_slices(g);
    hipLaunchKernelGGL(k_rho, dim3(((g.nx + 63) / 64) * nslice), dim3(kFT), 0, st, g, rho_part, rho_slices, nslice);
    return hipGetLastError();
}

hipError_t launch_species_rho(const Species* sp, int ns, int nx, int from_rho, double* rho_total, hipStream_t st)
{
    hipLaunchKernelGGL(k_species_rho, dim3((nx + 255) / 256), dim3(256), 0, st, sp, ns, nx, from_rho, rho_total);
    return hipGetLastError();
}

hipError_t launch_broadcast_E(const Species* sp, int ns, int nx, hipStream_t st)
{
    if (ns < 2) return hipSuccess;
    hipLaunchKernelGGL(k_broadcast_E, dim3((nx + 255) / 256), dim3(256), 0, st, sp, ns, nx);
    return hipGetLastError();
}

hipError_t launch_field(const Geo& g, const double* rho_part, const double* rho_in, double* rho_slices, double* rho,
                        double* E_out, const double2* tw, const double* green, double* diag_ring,
                        long long* step_ctr, int write_diag, double* W_out, int* flags, hipStream_t st)
{
    const size_t smem = (sizeof(double2) + sizeof(double2) / 2) * g.nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_solve, smem, granted);
    if (e != hipSuccess) return e;
    const int nslice = field_slices(g);
    if (!rho_in)
        hipLaunchKernelGGL(k_rho, dim3(((g.nx + 63) / 64) * nslice), dim3(kFT), 0, st, g, rho_part, rho_slices,
                           nslice);
    hipLaunchKernelGGL(k_solve, dim3(1), dim3(kFT), smem, st, g, rho_slices, nslice, rho_in, rho, E_out, tw, green,
                       diag_ring, step_ctr, write_diag, W_out, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// marker loading / export
// ---------------------------------------------------------------------------

// Check loaded FP64 markers: x in [0, L) and every value finite.
__global__ void k_validate(Geo g, const double* __restrict__ x, const double* __restrict__ v,
                           const double* __restrict__ f, int* __restrict__ bad)
{
    int local = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        const double xi = x[i];
        if (!(xi >= 0.0 && xi < g.L)) local = 1;
        if (!isfinite(f[i])) local = 1;
        for (int d = 0; d < g.vdim; ++d)
            if (!isfinite(v[(size_t)d * g.n + i])) local = 1;
    }
    if (local) atomicOr(bad, 1);
}

// FP64 markers -> FP32 form.
__global__ void k_to32(Geo g, const double* __restrict__ x, const double* __restrict__ v,
                       const double* __restrict__ f, M32 m, int* __restrict__ flags)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        double s = x[i] * g.inv_dx - 0.5;
        double fs = floor(s);
        float a = (float)(s - fs);
        int i0 = (int)fs;
        if (a >= 1.0f) { a = 0.0f; i0 += 1; }
        const int ix = i0 & (g.nx - 1);
        int jp[3];
        // velocity rows a cell index holds (the push clamps to the same range)
        const double lim = (double)(1 << (30 - g.lognx)) - 2.0;
        for (int d = 0; d < g.vdim; ++d) {
            double t = (v[(size_t)d * g.n + i] - g.vmin[d]) * g.inv_dv[d] - 0.5;
            double ft = floor(t);
            float b = (float)(t - ft);
            if (!(ft >= -lim && ft <= lim)) {
                // beyond what the form holds: clamped before the integer
                // conversion (which would overflow) and flagged
                atomicOr(flags, FLAG_RANGE);
                ft = fmin(fmax(ft, -lim), lim);
                b = 0.0f;
            }
            int j0 = (int)ft;
            if (b >= 1.0f) { b = 0.0f; j0 += 1; }
            m.b[(size_t)d * g.np + i] = b;
            jp[d] = j0 + 1;
        }
        int cell;
        if (g.vdim == 1) {
            cell = jp[0] * g.nx + ix;
        } else {
            int jj = jp[0] + g.jpad;
            const bool in_yz = jp[1] >= 0 && jp[1] <= g.nv[1] && jp[2] >= 0 && jp[2] <= g.nv[2];
            if (jj < 0 || jj >= g.jrange || !in_yz) {
                atomicOr(flags, FLAG_RANGE);
                jj = min(max(jj, 0), g.jrange - 1);
                if (!in_yz) {
                    // no cell index holds a vy or vz cloud off the grid: store
                    // one of the overflow bucket (vy, vz clamped, the x-velocity
                    // index below the grid), so that every kernel stays inside
                    // its arrays until the flag is reported
                    jp[1] = min(max(jp[1], 0), g.nv[1]);
                    jp[2] = min(max(jp[2], 0), g.nv[2]);
                    jj = 0;
                }
            }
            cell = ((jp[2] * (g.nv[1] + 1) + jp[1]) * g.jrange + jj) * g.nx + ix;
        }
        m.cell[i] = cell;
        m.a[i] = a;
        m.f[i] = (float)f[i];
    }
}

// FP32 form -> FP64 markers: x = (i0 + 1/2 + a) dx, v = vmin + (j0 + 1/2 + b) dv.
// Marker i goes to slot id[i] when id is given (identity order), else to
// slot i; f is written only when given.
__global__ void k_to64(Geo g, M32 m, double* __restrict__ x, double* __restrict__ v, double* __restrict__ f,
                       const int* __restrict__ id)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        const int o = id ? id[i] : i;
        const int cell = m.cell[i];
        const int ix = cell & (g.nx - 1);
        const int r = cell >> g.lognx;
        int jp[3];
        if (g.vdim == 1) {
            jp[0] = r;
        } else {
            jp[0] = (r & (g.jrange - 1)) - g.jpad;
            const int yz = r >> __builtin_ctz(g.jrange);
            jp[1] = yz % (g.nv[1] + 1);
            jp[2] = yz / (g.nv[1] + 1);
        }
        double xx = ((double)ix + 0.5 + (double)m.a[i]) * g.dx;
        if (xx >= g.L) xx -= g.L;
        x[o] = xx;
        for (int d = 0; d < g.vdim; ++d)
            v[(size_t)d * g.n + o] = g.vmin[d] + ((double)(jp[d] - 1) + 0.5 + (double)m.b[(size_t)d * g.np + i]) * g.dv[d];
        if (f) f[o] = (double)m.f[i];
    }
}

// Streaming copy: each thread moves four 16-byte vectors, all four loads
// issued before the stores.
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n16)
{
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t i = base + (size_t)k * 256;
        if (i < n16) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const size_t i = base + (size_t)k * 256;
        if (i < n16) dst[i] = v[k];
    }
}

hipError_t launch_validate(const Geo& g, const double* x, const double* v, const double* f, int* bad, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    int blocks = min((g.n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, st, g, x, v, f, bad);
    return hipGetLastError();
}

hipError_t launch_to32(const Geo& g, const double* x, const double* v, const double* f, M32 m, int* flags,
                       hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    int blocks = min((g.n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to32, dim3(blocks), dim3(256), 0, st, g, x, v, f, m, flags);
    return hipGetLastError();
}

hipError_t launch_to64(const Geo& g, M32 m, double* x, double* v, double* f, hipStream_t st, const int* id)
{
    if (g.n == 0) return hipSuccess;
    int blocks = min((g.n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to64, dim3(blocks), dim3(256), 0, st, g, m, x, v, f, id);
    return hipGetLastError();
}

// FP64 markers in identity order: x and v of marker i go to slot id[i].
__global__ void k_by_id64(int n, const double* __restrict__ x, const double* __restrict__ v,
                          const int* __restrict__ id, double* __restrict__ xo, double* __restrict__ vo)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int o = id[i];
        xo[o] = x[i];
        vo[o] = v[i];
    }
}

hipError_t launch_by_id64(int n, const double* x, const double* v, const int* id, double* xo, double* vo,
                          hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_by_id64, dim3(min((n + 255) / 256, 8192)), dim3(256), 0, st, n, x, v, id, xo, vo);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st)
{
    size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + 1023) / 1024;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)src, (float4*)dst, n16);
    return hipGetLastError();
}

}  // namespace avl
