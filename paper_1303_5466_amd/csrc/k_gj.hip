// Blocked Gauss-Jordan elimination without pivoting, batched over the boxes
// of a tree level.  Applied to the augmented block [F'_rr | F'_rs] it leaves
// G = (F'_rr)^{-1} in place of F'_rr and W = G F'_rs in place of F'_rs; the
// same routine inverts the top-level block (Algorithm 1, "direct inversion
// at the top level").  The matrices it is applied to are symmetric positive
// definite (Laplace) or identity-dominated complex symmetric (scattering),
// for which elimination in natural order is stable.
//
// One step handles a panel of nb pivot rows/columns:
//   pivot kernel  (this file): every workgroup inverts the nb x nb pivot
//                 block P in LDS, forms SR = P^{-1} X[piv, cols] for its own
//                 column chunk, zeroes X[piv, own cols], and the owner of a
//                 pivot column copies it to SC with -I in the pivot rows;
//   update        (grouped GEMM): X = X - SC * SR with beta = 0 on the pivot
//                 columns, which produces the new pivot rows (SR), the new
//                 pivot columns (-X_old[:, piv] P^{-1}) and the rank-nb update
//                 of everything else in one pass.
#include "common.hpp"

namespace rsd {

namespace {

constexpr int GJ_NB = 32;
constexpr int CHUNK = 64;

template <typename T>
__global__ void __launch_bounds__(256) gj_pivot_kernel(const GJDesc<T>* __restrict__ descs, int step,
                                                        int nb, int* __restrict__ err) {
    const GJDesc<T> d = descs[blockIdx.y];
    const int j0 = step * nb;
    if (j0 >= d.n) return;
    const int nbe = min(nb, d.n - j0);
    const int c_lo = blockIdx.x * CHUNK;
    if (c_lo >= d.ncols) return;
    const int t = threadIdx.x;
    __shared__ T P[GJ_NB][GJ_NB + 1];
    __shared__ T Xp[GJ_NB][CHUNK + 1];
    __shared__ T rowbuf[GJ_NB];
    __shared__ T colbuf[GJ_NB];
    __shared__ int bad;
    const int pc0 = d.pcol + j0;
    if (t == 0) bad = 0;
    for (int e = t; e < nbe * nbe; e += 256) {
        const int i = e % nbe, j = e / nbe;
        P[i][j] = d.X[(j0 + i) + (int64_t)(pc0 + j) * d.ld];
    }
    for (int e = t; e < nbe * CHUNK; e += 256) {
        const int q = e % nbe, cc = e / nbe;
        const int c = c_lo + cc;
        Xp[q][cc] = c < d.ncols ? d.X[(j0 + q) + (int64_t)c * d.ld] : T(0);
    }
    __syncthreads();
    // in-place inversion of P (natural order)
    for (int c = 0; c < nbe; ++c) {
        const T piv = P[c][c];
        if (t < nbe) {
            rowbuf[t] = (t == c ? T(1) : P[c][t]) / piv;
            colbuf[t] = P[t][c];
        }
        if (t == 0 && !(fabs((double)piv) > 1e-300 && isfinite((double)piv))) bad = 1;
        __syncthreads();
        for (int e = t; e < nbe * nbe; e += 256) {
            const int i = e % nbe, j = e / nbe;
            if (i == c) P[i][j] = rowbuf[j];
            else P[i][j] = (j == c ? T(0) : P[i][j]) - colbuf[i] * rowbuf[j];
        }
        __syncthreads();
    }
    if (t == 0 && bad && blockIdx.x == 0) atomicCAS(err, 0, d.box + 1);
    // SR for this column chunk, zero the pivot rows of non-pivot columns
    for (int e = t; e < nbe * CHUNK; e += 256) {
        const int q = e % nbe, cc = e / nbe;
        const int c = c_lo + cc;
        if (c >= d.ncols) continue;
        T v;
        if (c >= pc0 && c < pc0 + nbe) {
            v = P[q][c - pc0];
        } else {
            v = T(0);
            for (int s2 = 0; s2 < nbe; ++s2) v += P[q][s2] * Xp[s2][cc];
            d.X[(j0 + q) + (int64_t)c * d.ld] = T(0);
        }
        d.SR[q + (int64_t)c * nb] = v;
    }
    // owner of pivot columns: SC = old column, -I in the pivot rows
    const int lo = max(pc0, c_lo), hi = min(pc0 + nbe, min(c_lo + CHUNK, d.ncols));
    for (int c = lo; c < hi; ++c) {
        const int q = c - pc0;
        for (int i = t; i < d.n; i += 256) {
            T v;
            if (i >= j0 && i < j0 + nbe) v = (i - j0 == q) ? T(-1) : T(0);
            else v = d.X[i + (int64_t)c * d.ld];
            d.SC[i + (int64_t)q * d.n] = v;
        }
    }
}

}  // namespace

template <typename T>
void launch_gj_pivot(const GJDesc<T>* d, int n_desc, int step, int nb, int max_chunks, int* err,
                     hipStream_t s) {
    if (n_desc <= 0) return;
    hipLaunchKernelGGL(gj_pivot_kernel<T>, dim3(max_chunks, n_desc), dim3(256), 0, s, d, step, nb, err);
}

template void launch_gj_pivot<double>(const GJDesc<double>*, int, int, int, int, int*, hipStream_t);
template void launch_gj_pivot<float>(const GJDesc<float>*, int, int, int, int, int*, hipStream_t);

}  // namespace rsd
