// Reverse-mode (adjoint) kernels of the 1D-1V step (either storage form; the
// states are handed over as FP64 coordinates), for gradients of
// J = sum over steps n = 1..N of sum_i (E_i^n)^2 dx dt with respect to the
// marker weights f_l.
//
// Forward step n -> n+1 (Sec. 2): gather E at x^n with the cloud-in-cell
// weights, kick v, drift x; reconstruct f = N/D (Eq. (reconstruction)) from
// the pushed markers; rho_i = q dv sum_j f_ij; E = P rho with the spectral
// solve (Eq. (poissonk)).  Every stage is piecewise linear or rational in
// the marker coordinates (the sort only permutes), so the adjoint is the
// chain rule taken backwards:
//   * field:   rho_bar = P^T mu = -P mu (P is a real convolution with an odd
//              kernel: its transfer function -i c_p kappa/K^2 is odd and
//              imaginary);
//   * moments: f_bar_g = q dv rho_bar_i for every cell g of column i;
//   * f = N/D: N_bar = f_bar / D, D_bar = -f_bar f / D (cells with D = 0
//              carry nothing);
//   * deposit: a marker with weights alpha_c on its corners c gets
//              f_bar_l += sum_c alpha_c N_bar_c, and through d alpha/dx and
//              d alpha/dv position adjoints from G_c = N_bar_c f_l + D_bar_c;
//   * push:    x' = x + v' dt, v' = v + c E(x) with c = (q/m) dt (times the
//              kick fraction): lam_v <- lam_v' + lam_x' dt,
//              lam_x <- lam_x' + c E'(x) lam_v, E_bar(x) = c lam_v;
//   * gather:  mu_i^n += W_i(x^n) E_bar (deposited onto the grid).
// Adjoints are kept per marker identity (the sort moves identities with the
// markers), so recorded states can be visited in any order; the driver
// records states in identity order, so a reverse step reads coordinates,
// weights and adjoints at one index.  The gathered field adjoint is summed as
// integers (order-free), so the gradient is the same bit for bit from run to
// run.
#include <algorithm>

#include "avl_device.h"

namespace avl {

__global__ void k_iota(int* __restrict__ id, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) id[i] = i;
}

// Reverse of the reconstruction and moments for one marker at (x, v) with
// weight fl: its f_bar and the position adjoints dx, dv (per cell width).
// R times rscale is rho_bar (the driver passes P mu with rscale = -1); fg
// and Dg the state's grids.
template <typename T>
__device__ __forceinline__ void deposit_one(const Geo& g, double x, double v, double fl, const T* __restrict__ fg,
                                            const T* __restrict__ Dg, const double* __restrict__ R, double rscale,
                                            double& fb, double& dx, double& dv)
{
    const double s = x * g.inv_dx - 0.5;
    const double fs = floor(s);
    const double a = s - fs;
    const int ia = wrap_pow2((int)fs, g.nx);
    const int ib = wrap_pow2(ia + 1, g.nx);
    const double t = (v - g.vmin[0]) * g.inv_dv[0] - 0.5;
    const double ft = floor(t);
    const double b = t - ft;
    const int j0 = (int)ft;
    fb = 0.0;
    dx = 0.0;
    dv = 0.0;
#pragma unroll
    for (int cj = 0; cj < 2; ++cj) {
        const int j = j0 + cj;
        if (j < 0 || j >= g.nv[0]) continue;
        const double wy = cj ? b : 1.0 - b;
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
            const int col = ci ? ib : ia;
            const size_t gi = (size_t)j * g.nx + col;
            const double D = (double)Dg[gi];
            const double Nb = D > 0.0 ? rscale * g.q_vol * R[col] / D : 0.0;
            const double Db = -Nb * (double)fg[gi];
            const double G = Nb * fl + Db;
            const double wx = ci ? a : 1.0 - a;
            fb += wx * wy * Nb;
            dx += (ci ? wy : -wy) * G;
            dv += (cj ? wx : -wx) * G;
        }
    }
}

// Reverse of gather + kick + drift for one marker at x (its position before
// the push), E the field of that step: lam_v <- lam_v' + lam_x' dt,
// lam_x <- lam_x' + c E'(x) lam_v, in place on (Lx, Lv).
__device__ __forceinline__ void push_lam_one(const Geo& g, double x, const double* __restrict__ E, double c,
                                             double& Lx, double& Lv)
{
    const double lvt = Lv + Lx * g.dt;
    const double s = x * g.inv_dx - 0.5;
    const double fs = floor(s);
    const int ia = wrap_pow2((int)fs, g.nx);
    const int ib = wrap_pow2(ia + 1, g.nx);
    const double Ep = (E[ib] - E[ia]) * g.inv_dx;
    Lx = Lx + c * Ep * lvt;
    Lv = lvt;
}

// The largest key of a block into *key with one atomic (256 threads).
__device__ __forceinline__ void block_key_max(unsigned kmax, unsigned* __restrict__ key)
{
    __shared__ unsigned s_max[256 / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) kmax = max(kmax, (unsigned)__shfl_xor((int)kmax, off));
    if ((threadIdx.x & (kWave - 1)) == 0) s_max[threadIdx.x / kWave] = kmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = 0u;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) m = max(m, s_max[w]);
        if (m) atomicMax(key, m);
    }
}

// Reverse of the reconstruction and moments for the markers of one state.
// Marker k has identity id[k] (k itself when id is null); its adjoints are
// added at that identity.
template <typename T>
__global__ void k_adj_deposit(Geo g, const double* __restrict__ x, const double* __restrict__ v,
                              const int* __restrict__ id, const double* __restrict__ f_by_id,
                              const T* __restrict__ fg, const T* __restrict__ Dg,
                              const double* __restrict__ R, double rscale, double* __restrict__ lam_x,
                              double* __restrict__ lam_v, double* __restrict__ f_bar, int with_positions)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.n; k += gridDim.x * blockDim.x) {
        const int l = id ? id[k] : k;
        double fb, dx, dv;
        deposit_one<T>(g, x[k], v[k], f_by_id[l], fg, Dg, R, rscale, fb, dx, dv);
        f_bar[l] += fb;
        if (with_positions) {
            lam_x[l] += dx * g.inv_dx;
            lam_v[l] += dv * g.inv_dv[0];
        }
    }
}

// One reverse step for states recorded in identity order: the deposit
// reverse on the pushed state (x1, v1, its grids fg, Dg) followed, marker by
// marker, by the push reverse on the state before the push (x0, field E0) --
// the same arithmetic as k_adj_deposit then k_adj_push_lam, without storing
// and reloading the adjoints in between -- and the largest |c lam_v| into key.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_step_rev(Geo g, const double* __restrict__ x1,
                                                      const double* __restrict__ v1,
                                                      const double* __restrict__ f_by_id, const T* __restrict__ fg,
                                                      const T* __restrict__ Dg, const double* __restrict__ R,
                                                      double rscale, const double* __restrict__ x0,
                                                      const double* __restrict__ E0, double c,
                                                      double* __restrict__ lam_x, double* __restrict__ lam_v,
                                                      double* __restrict__ f_bar, unsigned* __restrict__ key)
{
    unsigned kmax = 0u;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.n; k += gridDim.x * blockDim.x) {
        double fb, dx, dv;
        deposit_one<T>(g, x1[k], v1[k], f_by_id[k], fg, Dg, R, rscale, fb, dx, dv);
        f_bar[k] += fb;
        double Lx = lam_x[k] + dx * g.inv_dx;
        double Lv = lam_v[k] + dv * g.inv_dv[0];
        push_lam_one(g, x0[k], E0, c, Lx, Lv);
        lam_x[k] = Lx;
        lam_v[k] = Lv;
        kmax = max(kmax, fix_key(c * Lv));
    }
    block_key_max(kmax, key);
}

// Order-free sums of the field adjoint E_bar.  Every term t of a launch is
// bounded by M < 2^(e + 1), e from the largest |E_bar| of the markers (found
// by the pass before).  The term is taken on the integer grid q = 2^(e+1-P):
// T = round(t / q), split as T = H 2^S + Lo with 0 <= Lo < 2^S, and H and Lo
// are summed in two 64-bit integers per column.  Integer sums do not depend
// on the order of their terms, so neither does E_bar; S = 62 - ceil(log2(n+1))
// and P = 2 S keep both sums of up to n terms inside int64, and each term is
// carried to M 2^-P.
struct DepScale {
    int S, P;
};

static DepScale dep_scale(int n)
{
    int lg = 0;
    while (lg < 62 && ((long long)1 << lg) < (long long)n + 1) ++lg;
    DepScale d;
    d.S = 62 - lg;
    d.P = 2 * d.S;
    return d;
}

__device__ __forceinline__ int dep_shift(unsigned key, int P)
{
    const int e = min(max(fix_exp_of_key(key, 0.0), -900), 1024);
    return P - e - 1;                        // q = 2^-shift
}

__device__ __forceinline__ void dep_add(unsigned long long* acc, int nx, int i, double t, int S, int shift)
{
    const double T = ldexp(t, shift);        // a power-of-two scaling: exact
    const double hf = floor(ldexp(T, -S));
    const long long H = (long long)hf;
    const long long Lo = (long long)rint(T - ldexp(hf, S));
    if (H) atomicAdd(&acc[i], (unsigned long long)H);
    if (Lo) atomicAdd(&acc[nx + i], (unsigned long long)Lo);
}

// Reverse of gather + kick + drift for the markers of state n (positions
// before the push), E the field at step n, first pass: the velocity and
// position adjoints (in place when the input and output arrays are the same),
// and the largest |c lam_v| of the launch into key.
__global__ __launch_bounds__(256) void k_adj_push_lam(Geo g, const double* __restrict__ x, const int* __restrict__ id,
                                                      const double* __restrict__ E, double c,
                                                      const double* lam_x_in, const double* lam_v_in,
                                                      double* lam_x, double* lam_v, unsigned* __restrict__ key)
{
    unsigned kmax = 0u;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.n; k += gridDim.x * blockDim.x) {
        const int l = id ? id[k] : k;
        double Lx = lam_x_in[l], Lv = lam_v_in[l];
        push_lam_one(g, x[k], E, c, Lx, Lv);
        lam_x[l] = Lx;
        lam_v[l] = Lv;
        kmax = max(kmax, fix_key(c * Lv));
    }
    // one atomic per block: the launch has a few blocks per CU, so the
    // single address sees a few thousand updates rather than one per wave
    block_key_max(kmax, key);
}

// Second pass: E_bar(x) = c lam_v gathered back onto the grid with the
// cloud-in-cell weights, (1-a) to column ia and a to ia + 1, as order-free
// integer sums, per block in LDS and then one global add per touched column.
// A block takes chunks of 8 markers a thread, blockIdx.x, blockIdx.x +
// gridDim.x, ...: markers in identity order reach every column from any
// chunk, so a bounded grid keeps the global adds to a few per column and block.
__global__ __launch_bounds__(256) void k_adj_push_dep(Geo g, const double* __restrict__ x, const int* __restrict__ id,
                                                      const double* __restrict__ lam_v, double c,
                                                      const unsigned* __restrict__ key, int S, int P,
                                                      unsigned long long* __restrict__ acc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* sacc = reinterpret_cast<unsigned long long*>(smem);
    const int nx = g.nx;
    for (int i = threadIdx.x; i < 2 * nx; i += blockDim.x) sacc[i] = 0ull;
    __syncthreads();
    const int shift = dep_shift(*key, P);
    const int per = blockDim.x * 8;
    for (int base = blockIdx.x * per; base < g.n; base += gridDim.x * per) {
        for (int k = base + threadIdx.x; k < min(base + per, g.n); k += blockDim.x) {
            const int l = id ? id[k] : k;
            const double Eb = c * lam_v[l];
            const double s = x[k] * g.inv_dx - 0.5;
            const double fs = floor(s);
            const double a = s - fs;
            const int ia = wrap_pow2((int)fs, nx);
            const int ib = wrap_pow2(ia + 1, nx);
            dep_add(sacc, nx, ia, (1.0 - a) * Eb, S, shift);
            dep_add(sacc, nx, ib, a * Eb, S, shift);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * nx; i += blockDim.x)
        if (sacc[i]) atomicAdd(&acc[i], sacc[i]);
}

// mu = w E + E_bar (w = 2 dx dt for a step that enters J; E may be null),
// with E_bar converted from its integer sums; the sums and the key are
// cleared for the next step.  One block.
__global__ __launch_bounds__(1024) void k_adj_mu(int nx, const double* __restrict__ E, double w, unsigned* key, int S,
                                                 int P, unsigned long long* __restrict__ acc, double* __restrict__ mu)
{
    const int shift = dep_shift(*key, P);
    __syncthreads();
    if (threadIdx.x == 0) *key = 0u;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const long long H = (long long)acc[i], Lo = (long long)acc[nx + i];
        const double dep = ldexp((double)H, S - shift) + ldexp((double)Lo, -shift);
        mu[i] = (E ? w * E[i] : 0.0) + dep;
        acc[i] = 0ull;
        acc[nx + i] = 0ull;
    }
}

__global__ void k_adj_clear(unsigned long long* __restrict__ acc, int nx, unsigned* __restrict__ key)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * nx; i += gridDim.x * blockDim.x) acc[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) *key = 0u;
}

__global__ void k_fill_f64(double* __restrict__ p, int n, double value)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = value;
}

__global__ void k_scale_f64(double* __restrict__ p, int n, double s)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] *= s;
}

static int grid_for(int n, int per) { return max(1, min((n + per - 1) / per, 8192)); }

hipError_t launch_iota(int* id, int n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, id, n);
    return hipGetLastError();
}

hipError_t launch_adj_deposit(const Geo& g, int grid_prec, const double* x, const double* v, const int* id,
                              const double* f_by_id, const void* fg, const void* Dg, const double* R, double rscale,
                              double* lam_x, double* lam_v, double* f_bar, int with_positions, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const dim3 gr(grid_for(g.n, 256)), bl(256);
    if (grid_prec == 0)
        hipLaunchKernelGGL(k_adj_deposit<double>, gr, bl, 0, st, g, x, v, id, f_by_id, (const double*)fg,
                           (const double*)Dg, R, rscale, lam_x, lam_v, f_bar, with_positions);
    else
        hipLaunchKernelGGL(k_adj_deposit<float>, gr, bl, 0, st, g, x, v, id, f_by_id, (const float*)fg,
                           (const float*)Dg, R, rscale, lam_x, lam_v, f_bar, with_positions);
    return hipGetLastError();
}

// acc: 2 nx unsigned 64-bit sums, key: one unsigned, both zero on entry (the
// clear below, then k_adj_mu leaves them zero).
hipError_t launch_adj_push(const Geo& g, const double* x, const int* id, const double* E, double c,
                           const double* lam_x_in, const double* lam_v_in, double* lam_x, double* lam_v,
                           unsigned long long* acc, unsigned* key, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const DepScale d = dep_scale(g.n);
    hipLaunchKernelGGL(k_adj_push_lam, dim3(std::min(grid_for(g.n, 256), 1024)), dim3(256), 0, st, g, x, id, E, c,
                       lam_x_in, lam_v_in, lam_x, lam_v, key);
    const size_t smem = sizeof(unsigned long long) * 2 * (size_t)g.nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_adj_push_dep, smem, granted);
    if (e != hipSuccess) return e;
    const int blocks = std::min((g.n + 256 * 8 - 1) / (256 * 8), 512);
    hipLaunchKernelGGL(k_adj_push_dep, dim3(blocks), dim3(256), smem, st, g, x, id, lam_v, c, key, d.S, d.P, acc);
    return hipGetLastError();
}

// One reverse step for states in identity order: k_adj_step_rev, then the
// field adjoint's integer deposit at the state before the push.
hipError_t launch_adj_step_rev(const Geo& g, int grid_prec, const double* x1, const double* v1, const double* f_by_id,
                               const void* fg, const void* Dg, const double* R, double rscale, const double* x0,
                               const double* E0, double c, double* lam_x, double* lam_v, double* f_bar,
                               unsigned long long* acc, unsigned* key, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    // enough blocks to keep the gathers in flight; one key atomic per block
    const dim3 gr(std::min(grid_for(g.n, 256), 4096)), bl(256);
    if (grid_prec == 0)
        hipLaunchKernelGGL(k_adj_step_rev<double>, gr, bl, 0, st, g, x1, v1, f_by_id, (const double*)fg,
                           (const double*)Dg, R, rscale, x0, E0, c, lam_x, lam_v, f_bar, key);
    else
        hipLaunchKernelGGL(k_adj_step_rev<float>, gr, bl, 0, st, g, x1, v1, f_by_id, (const float*)fg,
                           (const float*)Dg, R, rscale, x0, E0, c, lam_x, lam_v, f_bar, key);
    const DepScale d = dep_scale(g.n);
    const size_t smem = sizeof(unsigned long long) * 2 * (size_t)g.nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_adj_push_dep, smem, granted);
    if (e != hipSuccess) return e;
    const int blocks = std::min((g.n + 256 * 8 - 1) / (256 * 8), 512);
    hipLaunchKernelGGL(k_adj_push_dep, dim3(blocks), dim3(256), smem, st, g, x0, nullptr, lam_v, c, key, d.S, d.P,
                       acc);
    return hipGetLastError();
}

hipError_t launch_adj_mu(const Geo& g, const double* E, double w, unsigned long long* acc, unsigned* key, double* mu,
                         hipStream_t st)
{
    const DepScale d = dep_scale(g.n);
    hipLaunchKernelGGL(k_adj_mu, dim3(1), dim3(1024), 0, st, g.nx, E, w, key, d.S, d.P, acc, mu);
    return hipGetLastError();
}

hipError_t launch_adj_clear(int nx, unsigned long long* acc, unsigned* key, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_clear, dim3(grid_for(2 * nx, 256)), dim3(256), 0, st, acc, nx, key);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int n, double value, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_scale_f64(double* p, int n, double s, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_f64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, s);
    return hipGetLastError();
}

}  // namespace avl
