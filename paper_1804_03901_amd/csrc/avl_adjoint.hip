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
// markers), so recorded states can be visited in any order.
#include "avl_device.h"

namespace avl {

__global__ void k_iota(int* __restrict__ id, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) id[i] = i;
}

// Reverse of the reconstruction and moments for the markers of one state:
// Pmu = P mu (so rho_bar = -Pmu), fg and Dg the state's grids.
template <typename T>
__global__ void k_adj_deposit(Geo g, const double* __restrict__ x, const double* __restrict__ v,
                              const int* __restrict__ id, const double* __restrict__ f_by_id,
                              const T* __restrict__ fg, const T* __restrict__ Dg,
                              const double* __restrict__ Pmu, double* __restrict__ lam_x,
                              double* __restrict__ lam_v, double* __restrict__ f_bar, int with_positions)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.n; k += gridDim.x * blockDim.x) {
        const int l = id[k];
        const double fl = f_by_id[l];
        const double s = x[k] * g.inv_dx - 0.5;
        const double fs = floor(s);
        const double a = s - fs;
        const int ia = wrap_pow2((int)fs, g.nx);
        const int ib = wrap_pow2(ia + 1, g.nx);
        const double t = (v[k] - g.vmin[0]) * g.inv_dv[0] - 0.5;
        const double ft = floor(t);
        const double b = t - ft;
        const int j0 = (int)ft;
        double fb = 0.0, dx = 0.0, dv = 0.0;
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
                const double Nb = D > 0.0 ? -g.q_vol * Pmu[col] / D : 0.0;
                const double Db = -Nb * (double)fg[gi];
                const double G = Nb * fl + Db;
                const double wx = ci ? a : 1.0 - a;
                fb += wx * wy * Nb;
                dx += (ci ? wy : -wy) * G;
                dv += (cj ? wx : -wx) * G;
            }
        }
        f_bar[l] += fb;
        if (with_positions) {
            lam_x[l] += dx * g.inv_dx;
            lam_v[l] += dv * g.inv_dv[0];
        }
    }
}

// Reverse of gather + kick + drift for the markers of state n (positions
// before the push), E the field at step n.  The field adjoint is summed per
// block in LDS and added to mu_dep with one FP64 atomic per touched column.
__global__ __launch_bounds__(256) void k_adj_push(Geo g, const double* __restrict__ x, const int* __restrict__ id,
                                                  const double* __restrict__ E, double c,
                                                  double* __restrict__ lam_x, double* __restrict__ lam_v,
                                                  double* __restrict__ mu_dep)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* dep = reinterpret_cast<double*>(smem);
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) dep[i] = 0.0;
    __syncthreads();
    const int per = blockDim.x * 8;
    const int base = blockIdx.x * per;
    for (int k = base + threadIdx.x; k < min(base + per, g.n); k += blockDim.x) {
        const int l = id[k];
        const double Lx = lam_x[l], Lv = lam_v[l];
        const double lvt = Lv + Lx * g.dt;
        const double s = x[k] * g.inv_dx - 0.5;
        const double fs = floor(s);
        const double a = s - fs;
        const int ia = wrap_pow2((int)fs, g.nx);
        const int ib = wrap_pow2(ia + 1, g.nx);
        const double Ep = (E[ib] - E[ia]) * g.inv_dx;
        lam_x[l] = Lx + c * Ep * lvt;
        lam_v[l] = lvt;
        const double Eb = c * lvt;
        atomicAdd(&dep[ia], (1.0 - a) * Eb);
        atomicAdd(&dep[ib], a * Eb);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x)
        if (dep[i] != 0.0) atomicAdd(&mu_dep[i], dep[i]);
}

// mu = w * E + mu_dep (w = 2 dx dt for a step that enters J, else 0); mu_dep
// is cleared for the next step.
__global__ void k_adj_mu(int nx, const double* __restrict__ E, double w, double* __restrict__ mu_dep,
                         double* __restrict__ mu)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += gridDim.x * blockDim.x) {
        mu[i] = w * E[i] + mu_dep[i];
        mu_dep[i] = 0.0;
    }
}

static int grid_for(int n, int per) { return max(1, min((n + per - 1) / per, 8192)); }

hipError_t launch_iota(int* id, int n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, st, id, n);
    return hipGetLastError();
}

hipError_t launch_adj_deposit(const Geo& g, int grid_prec, const double* x, const double* v, const int* id,
                              const double* f_by_id, const void* fg, const void* Dg, const double* Pmu, double* lam_x,
                              double* lam_v, double* f_bar, int with_positions, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const dim3 gr(grid_for(g.n, 256)), bl(256);
    if (grid_prec == 0)
        hipLaunchKernelGGL(k_adj_deposit<double>, gr, bl, 0, st, g, x, v, id, f_by_id, (const double*)fg,
                           (const double*)Dg, Pmu, lam_x, lam_v, f_bar, with_positions);
    else
        hipLaunchKernelGGL(k_adj_deposit<float>, gr, bl, 0, st, g, x, v, id, f_by_id, (const float*)fg,
                           (const float*)Dg, Pmu, lam_x, lam_v, f_bar, with_positions);
    return hipGetLastError();
}

hipError_t launch_adj_push(const Geo& g, const double* x, const int* id, const double* E, double c, double* lam_x,
                           double* lam_v, double* mu_dep, hipStream_t st)
{
    if (g.n == 0) return hipSuccess;
    const size_t smem = sizeof(double) * g.nx;
    static int granted = 0;
    hipError_t e = ensure_lds((const void*)k_adj_push, smem, granted);
    if (e != hipSuccess) return e;
    const int blocks = (g.n + 256 * 8 - 1) / (256 * 8);
    hipLaunchKernelGGL(k_adj_push, dim3(blocks), dim3(256), smem, st, g, x, id, E, c, lam_x, lam_v, mu_dep);
    return hipGetLastError();
}

hipError_t launch_adj_mu(int nx, const double* E, double w, double* mu_dep, double* mu, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_mu, dim3(grid_for(nx, 256)), dim3(256), 0, st, nx, E, w, mu_dep, mu);
    return hipGetLastError();
}

}  // namespace avl
