// Exact float64 product y = A x for the Nystrom matrix on the grid (Sec. 5,
// general formulation), used for residuals of iterative refinement.
//
// The off-diagonal part of A depends only on the grid offset, so one table
// Kt[|di|][|dj|] = h^2 K(h |(di, dj)|) (N entries) replaces every kernel
// evaluation.  Each workgroup owns a 16 x 16 tile of targets and sweeps all
// 16 x 16 source tiles; the 31 x 31 window of the table the tile pair needs
// and the source values are staged in LDS.  Direct summation: every pair is
// visited once, in a fixed order, so results are deterministic.
#include "common.hpp"

namespace rsd {

namespace {

constexpr double INV_2PI = 0.15915494309189533576888376337251;
constexpr int TS = 16;
constexpr int RC = 8;   // right-hand sides per pass

__global__ void table_kernel(double* __restrict__ Kt, int64_t nx, int64_t ny, KernelDesc kd) {
    const int64_t n = nx * ny;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t di = e / ny, dj = e % ny;
        double v = 0.0;
        if (e != 0) v = kd.h * kd.h * INV_2PI * (kd.logh + 0.5 * log((double)(di * di + dj * dj)));
        Kt[e] = v;
    }
}

__global__ void __launch_bounds__(256) matvec_kernel(double* __restrict__ y,
                                                     const double* __restrict__ x, int nrhs,
                                                     const double* __restrict__ Kt, int64_t nx,
                                                     int64_t ny, KernelDesc kd) {
    __shared__ double W[2 * TS - 1][2 * TS];
    __shared__ double xs[TS * TS][RC];
    const int tl = threadIdx.x;
    const int til = tl / TS, tjl = tl % TS;
    const int64_t ti0 = (int64_t)blockIdx.x * TS, tj0 = (int64_t)blockIdx.y * TS;
    const int64_t ti = ti0 + til, tj = tj0 + tjl;
    const bool valid = ti < nx && tj < ny;
    const int64_t N = nx * ny;
    for (int c0 = 0; c0 < nrhs; c0 += RC) {
        const int nc = min(RC, nrhs - c0);
        double acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = 0.0;
        for (int64_t si0 = 0; si0 < nx; si0 += TS) {
            for (int64_t sj0 = 0; sj0 < ny; sj0 += TS) {
                __syncthreads();
                const int64_t D0i = ti0 - si0 - (TS - 1), D0j = tj0 - sj0 - (TS - 1);
                for (int e = tl; e < (2 * TS - 1) * (2 * TS - 1); e += 256) {
                    const int wi = e / (2 * TS - 1), wj = e % (2 * TS - 1);
                    int64_t di = D0i + wi, dj = D0j + wj;
                    di = di < 0 ? -di : di;
                    dj = dj < 0 ? -dj : dj;
                    W[wi][wj] = (di < nx && dj < ny) ? Kt[di * ny + dj] : 0.0;
                }
                {
                    const int64_t si = si0 + til, sj = sj0 + tjl;
                    const bool sv = si < nx && sj < ny;
                    double sb = 1.0;
                    if (sv && kd.has_b) sb = kd.sb[si * ny + sj];
#pragma unroll
                    for (int c = 0; c < RC; ++c)
                        xs[tl][c] = (sv && c < nc) ? sb * x[(si * ny + sj) + (int64_t)(c0 + c) * N] : 0.0;
                }
                __syncthreads();
                if (valid) {
                    for (int s = 0; s < TS * TS; ++s) {
                        const int sil = s / TS, sjl = s % TS;
                        const double w = W[til - sil + TS - 1][tjl - sjl + TS - 1];
#pragma unroll
                        for (int c = 0; c < RC; ++c) acc[c] += w * xs[s][c];
                    }
                }
            }
        }
        if (valid) {
            const int64_t g = ti * ny + tj;
            double dg, sb = 1.0;
            if (kd.has_b) { sb = kd.sb[g]; dg = 1.0 + sb * sb * kd.sc_re; }
            else dg = (kd.a ? kd.a[g] : 1.0) + kd.sc_re;
            for (int c = 0; c < nc; ++c)
                y[g + (int64_t)(c0 + c) * N] = sb * acc[c] + dg * x[g + (int64_t)(c0 + c) * N];
        }
    }
}

}  // namespace

void launch_matvec_table(double* table, int64_t nx, int64_t ny, KernelDesc kd, hipStream_t s) {
    int64_t blocks = (nx * ny + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(table_kernel, dim3((int)blocks), dim3(256), 0, s, table, nx, ny, kd);
}

void launch_matvec(double* y, const double* x, int nrhs, const double* table, int64_t nx,
                   int64_t ny, KernelDesc kd, int cplx, hipStream_t s) {
    if (cplx) throw HipError("complex matvec not available");
    dim3 grid((unsigned)((nx + TS - 1) / TS), (unsigned)((ny + TS - 1) / TS));
    hipLaunchKernelGGL(matvec_kernel, grid, dim3(256), 0, s, y, x, nrhs, table, nx, ny, kd);
}

}  // namespace rsd
