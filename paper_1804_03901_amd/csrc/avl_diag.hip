// Thermodynamic and field diagnostics of the reconstructed state (the
// quantities the paper writes per output step, Sec. 3.4): field energy, kinetic
// energy, their sum, the integral of f (number of particles), the integral of
// f log f (coarse-grained entropy, as the paper defines it), the momentum, the
// current density j(x), and the field solver's residual charge
// rho - dE/dx / c_p with a centred difference for the divergence.
//
// The f grid is read once: one thread per x column walks a chunk of velocity
// rows (coalesced across the block, x fastest in the grid) and writes four
// per-(chunk, column) partial sums; one block then adds the chunks per column
// in chunk order and the columns in a fixed tree, so every result has a fixed
// summation order.  All sums are FP64 (the FP32 form's grid is widened).
#include <algorithm>

#include "avl_device.h"

namespace avl {

// velocity rows (product of the velocity cell counts) of a geometry
__host__ __device__ inline long long diag_rows(const Geo& g)
{
    long long r = 1;
    for (int d = 0; d < g.vdim; ++d) r *= g.nv[d];
    return r;
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_part(Geo g, const T* __restrict__ f, int rows_per_chunk,
                                                            double* __restrict__ part)
{
    const int i = blockIdx.x * kDiagThreads + threadIdx.x;
    const int chunk = blockIdx.y;
    if (i >= g.nx) return;
    const long long rows = diag_rows(g);
    const long long r0 = (long long)chunk * rows_per_chunk;
    const long long r1 = min(r0 + rows_per_chunk, rows);
    const int nvx = g.nv[0];
    const int nvy = g.vdim == 3 ? g.nv[1] : 1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, sl = 0.0;
    for (long long r = r0; r < r1; ++r) {
        const double fv = (double)f[r * g.nx + i];
        const int jx = (int)(r % nvx);
        const double vx = g.vmin[0] + (jx + 0.5) * g.dv[0];
        double v2 = vx * vx;
        if (g.vdim == 3) {
            const long long q = r / nvx;
            const int jy = (int)(q % nvy);
            const int jz = (int)(q / nvy);
            const double vy = g.vmin[1] + (jy + 0.5) * g.dv[1];
            const double vz = g.vmin[2] + (jz + 0.5) * g.dv[2];
            v2 = (v2 + vy * vy) + vz * vz;
        }
        s0 += fv;
        s1 += fv * vx;
        s2 += fv * v2;
        if (fv > 0.0) sl += fv * log(fv);
    }
    const size_t stride = (size_t)gridDim.y * g.nx;
    const size_t o = (size_t)chunk * g.nx + i;
    part[o] = s0;
    part[stride + o] = s1;
    part[2 * stride + o] = s2;
    part[3 * stride + o] = sl;
}

// One block: per column, the chunk partials in chunk order; then the column
// sums in a fixed tree.  out = {Ee, Ekin, Etot, N, S, P}; j and drho per x
// (either may be null).
__global__ __launch_bounds__(kFieldThreads) void k_diag_final(Geo g, const double* __restrict__ part, int nchunk,
                                                              const double* __restrict__ rho,
                                                              const double* __restrict__ E, double mass,
                                                              double* __restrict__ out, double* __restrict__ j_out,
                                                              double* __restrict__ drho_out)
{
    constexpr int Q = 6;   // sum f, sum f v_x, sum f |v|^2, sum f log f, sum rho, sum E^2
    __shared__ double red[Q][kFieldThreads];
    const int t = threadIdx.x;
    double vol = g.dx;
    for (int d = 0; d < g.vdim; ++d) vol *= g.dv[d];
    const size_t stride = (size_t)nchunk * g.nx;
    double acc[Q] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = t; i < g.nx; i += kFieldThreads) {
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, cl = 0.0;
        for (int k = 0; k < nchunk; ++k) {
            const size_t o = (size_t)k * g.nx + i;
            c0 += part[o];
            c1 += part[stride + o];
            c2 += part[2 * stride + o];
            cl += part[3 * stride + o];
        }
        if (j_out) j_out[i] = g.q_vol * c1;   // q * prod(dv) * sum_j v_x f
        acc[0] += c0;
        acc[1] += c1;
        acc[2] += c2;
        acc[3] += cl;
        acc[4] += rho[i];
        acc[5] += E[i] * E[i];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) red[q][t] = acc[q];
    __syncthreads();
    for (int h = kFieldThreads / 2; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < Q; ++q) red[q][t] = red[q][t] + red[q][t + h];
        __syncthreads();
    }
    if (drho_out) {
        // the neutralising background is minus the mean charge density
        const double rho_mean = red[4][0] / g.nx;
        const double inv = 1.0 / (2.0 * g.dx * g.cp);
        for (int i = t; i < g.nx; i += kFieldThreads) {
            const double div = (E[(i + 1) & (g.nx - 1)] - E[(i - 1) & (g.nx - 1)]) * inv;
            drho_out[i] = (rho[i] - rho_mean) - div;
        }
    }
    if (t == 0) {
        const double Ee = red[5][0] * g.dx / (2.0 * g.cp);
        const double Ekin = 0.5 * mass * red[2][0] * vol;
        out[0] = Ee;
        out[1] = Ekin;
        out[2] = Ee + Ekin;
        out[3] = red[0][0] * vol;
        out[4] = red[3][0] * vol;
        out[5] = mass * red[1][0] * vol;
    }
}

int diag_chunks(const Geo& g)
{
    const int gx = (g.nx + kDiagThreads - 1) / kDiagThreads;
    const long long rows = diag_rows(g);
    return (int)std::max<long long>(1, std::min<long long>(rows, std::max(1, kDiagBlocks / gx)));
}

hipError_t launch_diag(const Geo& g, const void* fgrid, const double* rho, const double* E, double mass,
                       double* part, double* out, double* j_out, double* drho_out, hipStream_t st)
{
    const int nchunk = diag_chunks(g);
    const long long rows = diag_rows(g);
    const int rpc = (int)((rows + nchunk - 1) / nchunk);
    const dim3 gr((g.nx + kDiagThreads - 1) / kDiagThreads, nchunk);
    if (g.prec == 0)
        hipLaunchKernelGGL(k_diag_part<double>, gr, dim3(kDiagThreads), 0, st, g, (const double*)fgrid, rpc, part);
    else
        hipLaunchKernelGGL(k_diag_part<float>, gr, dim3(kDiagThreads), 0, st, g, (const float*)fgrid, rpc, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kFieldThreads), 0, st, g, (const double*)part, nchunk, rho, E, mass,
                       out, j_out, drho_out);
    return hipGetLastError();
}

}  // namespace avl
