// Charge density, spectral field solve and per-step diagnostics, one block.
//
// rho_i = q * prod(dv) * sum_j f_ij is assembled from the reconstruction's
// per-chunk column partials in chunk order (Sec. 2: the moment is a plain sum
// over velocity cells at fixed x).  The field follows Eq. (poissonk) with the
// softening of Eq. (kappasoftening): a radix-2 FFT of rho in LDS (decimation in
// time from bit-reversed order), multiplication by -i c_p kappa_m / K_m^2 (a
// host-built table that is zero at m = 0 and at the Nyquist mode), and an
// inverse FFT (decimation in frequency, natural order in, bit-reversed out).
// nx <= 4096 complex doubles fit in 64 KB of LDS.  The whole solve is FP64.
// Also here: marker validation/conversion kernels and the copy probe.
#include "avl_device.h"

namespace avl {

static int g_lds_limit = 65536;
void set_lds_limit(int bytes) { g_lds_limit = bytes; }
int lds_limit() { return g_lds_limit; }

__device__ __forceinline__ int bitrev(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int NT>
__device__ void block_sum3(double& a, double& b, double& c, double* s)
{
    s[threadIdx.x] = a;
    s[NT + threadIdx.x] = b;
    s[2 * NT + threadIdx.x] = c;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[threadIdx.x] += s[threadIdx.x + o];
            s[NT + threadIdx.x] += s[NT + threadIdx.x + o];
            s[2 * NT + threadIdx.x] += s[2 * NT + threadIdx.x + o];
        }
        __syncthreads();
    }
    a = s[0];
    b = s[NT];
    c = s[2 * NT];
}

// One launch for the charge density and the field.  Every block assembles rho
// for 64 x cells from the reconstruction's chunk partials (four groups of
// chunks per column, combined in a fixed order), then the last block to
// finish -- found with a device-scope fence and a counter it resets -- runs
// the FFT solve.  With rho given by the caller a single block does the solve.
__global__ __launch_bounds__(kFieldThreads) void k_field(Geo g, const double* __restrict__ rho_part,
                                                         const double* __restrict__ rho_in,
                                                         double* __restrict__ rho, double* __restrict__ E_out,
                                                         const double2* __restrict__ tw,
                                                         const double* __restrict__ green,
                                                         double* __restrict__ diag_ring,
                                                         long long* __restrict__ step_ctr, int write_diag,
                                                         double* __restrict__ W_out, int* __restrict__ flags,
                                                         int* __restrict__ done)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = g.nx, lg = g.lognx;
    const int half_n = nx >> 1;
    double2* z = reinterpret_cast<double2*>(smem);
    double2* stw = z + nx;
    double* sgr = reinterpret_cast<double*>(stw + half_n);
    __shared__ double red[3 * kFieldThreads];
    __shared__ int s_last;
    const double* src = rho_in;

    if (!rho_in) {
        // rho_i = q prod(dv) sum_c part[c][i]
        double* colsum = red;   // [4][64]
        const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
        const int i = blockIdx.x * 64 + c;
        double acc = 0.0;
        if (i < nx) {
            // batches of 16 independent loads (chunks grp, grp+4, ...), summed in order
            for (int ch0 = grp; ch0 < g.nchunk; ch0 += 64) {
                double v[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int ch = ch0 + 4 * k;
                    v[k] = ch < g.nchunk ? rho_part[(size_t)ch * nx + i] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) acc += v[k];
            }
        }
        colsum[grp * 64 + c] = acc;
        __syncthreads();
        if (grp == 0 && i < nx)
            rho[i] = (((colsum[c] + colsum[64 + c]) + colsum[128 + c]) + colsum[192 + c]) * g.q_vol;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) s_last = atomicAdd(done, 1) == (int)gridDim.x - 1;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        src = rho;
    }

    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        z[bitrev(i, lg)] = make_double2(src[i], 0.0);
        sgr[i] = green[i];
        if (i < half_n) stw[i] = tw[i];
    }
    __syncthreads();
    // forward transform, rho_hat_m = sum_i rho_i exp(-2 pi i m i / nx)
    for (int lh = 0; (1 << lh) < nx; ++lh) {
        const int half = 1 << lh, len = half << 1, stride = nx / len;
        for (int b = threadIdx.x; b < half_n; b += blockDim.x) {
            const int grp = b >> lh, p = b & (half - 1);
            const int i0 = grp * len + p, i1 = i0 + half;
            const double2 t = cmul(stw[p * stride], z[i1]);
            const double2 u = z[i0];
            z[i0] = make_double2(u.x + t.x, u.y + t.y);
            z[i1] = make_double2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
    // E_hat_m = -i * (c_p kappa_m / K_m^2) * rho_hat_m
    for (int m = threadIdx.x; m < nx; m += blockDim.x) {
        const double2 r = z[m];
        const double c = sgr[m];
        z[m] = make_double2(c * r.y, -c * r.x);
    }
    __syncthreads();
    // inverse transform (unnormalised), natural order in, bit-reversed out
    for (int lh = lg - 1; lh >= 0; --lh) {
        const int half = 1 << lh, len = half << 1, stride = nx / len;
        for (int b = threadIdx.x; b < half_n; b += blockDim.x) {
            const int grp = b >> lh, p = b & (half - 1);
            const int i0 = grp * len + p, i1 = i0 + half;
            const double2 u = z[i0], v = z[i1];
            const double2 w = stw[p * stride];
            z[i0] = make_double2(u.x + v.x, u.y + v.y);
            z[i1] = cmul(make_double2(u.x - v.x, u.y - v.y), make_double2(w.x, -w.y));
        }
        __syncthreads();
    }
    double sw = 0.0, sre = 0.0, sim = 0.0;
    int bad = 0;
    const double inv_n = 1.0 / nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double E = z[bitrev(i, lg)].x * inv_n;
        E_out[i] = E;
        if (!isfinite(E)) bad = 1;
        sw += E * E;
        const double2 w = i < half_n ? stw[i] : make_double2(-stw[i - half_n].x, -stw[i - half_n].y);
        sre += E * w.x;
        sim += E * w.y;
    }
    if (bad) atomicOr(flags, FLAG_NONFINITE);
    __syncthreads();
    block_sum3<kFieldThreads>(sw, sre, sim, red);
    if (threadIdx.x == 0) {
        const double W = sw * g.dx / (2.0 * g.cp);
        const double m1 = 2.0 / nx * sqrt(sre * sre + sim * sim);
        if (W_out) *W_out = W;
        if (write_diag) {
            const long long c = *step_ctr;
            diag_ring[2 * (c % kDiagCap)] = W;
            diag_ring[2 * (c % kDiagCap) + 1] = m1;
            *step_ctr = c + 1;
        }
        if (!rho_in) *done = 0;
    }
}

hipError_t launch_field(const Geo& g, const double* rho_part, const double* rho_in, double* rho, double* E_out,
                        const double2* tw, const double* green, double* diag_ring, long long* step_ctr,
                        int write_diag, double* W_out, int* flags, int* done, hipStream_t st)
{
    const size_t smem = (sizeof(double2) + sizeof(double2) / 2 + sizeof(double)) * g.nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_field, smem, granted);
    if (e != hipSuccess) return e;
    const int blocks = rho_in ? 1 : (g.nx + 63) / 64;
    hipLaunchKernelGGL(k_field, dim3(blocks), dim3(kFieldThreads), smem, st, g, rho_part, rho_in, rho, E_out, tw,
                       green, diag_ring, step_ctr, write_diag, W_out, flags, done);
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
        for (int d = 0; d < g.vdim; ++d) {
            double t = (v[(size_t)d * g.n + i] - g.vmin[d]) * g.inv_dv[d] - 0.5;
            double ft = floor(t);
            float b = (float)(t - ft);
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
            if (jj < 0 || jj >= g.jrange || jp[1] < 0 || jp[1] > g.nv[1] || jp[2] < 0 || jp[2] > g.nv[2]) {
                atomicOr(flags, FLAG_RANGE);
                jj = min(max(jj, 0), g.jrange - 1);
            }
            cell = ((jp[2] * (g.nv[1] + 1) + jp[1]) * g.jrange + jj) * g.nx + ix;
        }
        m.cell[i] = cell;
        m.a[i] = a;
        m.f[i] = (float)f[i];
    }
}

// FP32 form -> FP64 markers: x = (i0 + 1/2 + a) dx, v = vmin + (j0 + 1/2 + b) dv.
__global__ void k_to64(Geo g, M32 m, double* __restrict__ x, double* __restrict__ v, double* __restrict__ f)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x) {
        const int cell = m.cell[i];
        const int ix = cell & (g.nx - 1);
        const int r = cell >> g.lognx;
        int jp[3];
        if (g.vdim == 1) {
            jp[0] = r;
        } else {
            jp[0] = (r % g.jrange) - g.jpad;
            const int yz = r / g.jrange;
            jp[1] = yz % (g.nv[1] + 1);
            jp[2] = yz / (g.nv[1] + 1);
        }
        double xx = ((double)ix + 0.5 + (double)m.a[i]) * g.dx;
        if (xx >= g.L) xx -= g.L;
        x[i] = xx;
        for (int d = 0; d < g.vdim; ++d)
            v[(size_t)d * g.n + i] = g.vmin[d] + ((double)(jp[d] - 1) + 0.5 + (double)m.b[(size_t)d * g.np + i]) * g.dv[d];
        f[i] = (double)m.f[i];
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

hipError_t launch_to64(const Geo& g, M32 m, double* x, double* v, double* f, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    int blocks = min((g.n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_to64, dim3(blocks), dim3(256), 0, st, g, m, x, v, f);
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
