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

constexpr int GJ_NB = 64;
constexpr int CHUNK = 64;

// Buffer loads from the matrix with 32-bit byte offsets from descriptors based
// at the pivot block and at the work-group's column chunk (the host keeps the
// 64 columns such a descriptor reaches below GJ_RSRC_RANGE bytes); the offset
// GJ_RSRC_RANGE itself is out of range and reads zero.
constexpr int GJ_RSRC_RANGE = 0x7ffffff0;
constexpr int GJ_RSRC_WORD3 = 0x00020000;    // raw buffer, 32-bit data format

template <typename T> __device__ inline T gj_load(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ inline double gj_load<double>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ inline float gj_load<float>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// MFMA 16x16x4 called with its operands swapped, step(b, a, acc): element
// v of lane l is then C[l % 16][col(l, v)] of the product C = A B, where
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
typedef double gj_d4 __attribute__((ext_vector_type(4)));
typedef float gj_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct GjMfma;
template <> struct GjMfma<double> {
    typedef gj_d4 acc_t;
    __device__ static inline int col(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct GjMfma<float> {
    typedef gj_f4 acc_t;
    __device__ static inline int col(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// 1 / x from the hardware reciprocal estimate and two Newton steps (each
// squares the relative error), shorter than an IEEE division on the
// elimination's critical path; x is a checked, normal pivot.
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}
__device__ inline float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// Inversion of the pivot block: thread t keeps the 4 x 4 tile (rows 4(t/16),
// columns 4(t%16)) of P in registers; step c needs only pivot row c and pivot
// column c, which their owners publish in a double-buffered LDS strip, so each
// elimination step costs one barrier.  The step is straight-line code: every
// element computes the generic update and selects the pivot-row/column forms.
//
// PAIR (complex factors, whose dofs come in adjacent pairs forming the 2 x 2
// real form [[re, im], [im, -re]] of a complex entry): the steps eliminate
// two pivots at a time with the inverse of their 2 x 2 block, so that the
// pivot is the complex entry (determinant -|z|^2) and never its real part
// alone, which vanishes where the Schur complements turn (interpolation
// matrices of boxes about a wavelength across).
template <typename T, bool PAIR>
__global__ void __launch_bounds__(256) gj_pivot_kernel(const GJDesc<T>* __restrict__ descs, int step,
                                                        int nb, int* __restrict__ err) {
    const GJDesc<T> d = descs[blockIdx.y];
    const int j0 = step * nb;
    if (j0 >= d.n) return;
    const int nbe = min(nb, d.n - j0);
    const int c_lo = blockIdx.x * CHUNK;
    if (c_lo >= d.ncols) return;
    const int t = threadIdx.x;
    const int ri = 4 * (t >> 4), cj = 4 * (t & 15);
    __shared__ T Pi[GJ_NB][GJ_NB + 1];
    __shared__ T Xp[GJ_NB][CHUNK + 1];
    // published pivot rows / columns, double buffered (PAIR: two of each)
    __shared__ __align__(16) T rowb[2][PAIR ? 2 : 1][GJ_NB];
    __shared__ __align__(16) T colb[2][PAIR ? 2 : 1][GJ_NB];
    __shared__ int bad;
    const int pc0 = d.pcol + j0;
    // every load of the pivot block and of the chunk's pivot rows is issued
    // before the first is used: buffer loads, masked by an out-of-range offset
    // (which reads zero), so that no branch separates them
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(d.X + j0 + (int64_t)pc0 * d.ld), (short)0, GJ_RSRC_RANGE, GJ_RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(d.X + j0 + (int64_t)c_lo * d.ld), (short)0, GJ_RSRC_RANGE, GJ_RSRC_WORD3);
    T p[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ri + a, j = cj + b;
            const bool ok = (i < nbe) & (j < nbe);
            p[a][b] = gj_load<T>(rp, ok ? (i + j * d.ld) * (int)sizeof(T) : GJ_RSRC_RANGE);
        }
    T xv[GJ_NB * CHUNK / 256];
#pragma unroll
    for (int u = 0; u < GJ_NB * CHUNK / 256; ++u) {
        const int e = t + 256 * u;
        const int q = e & (GJ_NB - 1), c = c_lo + e / GJ_NB;
        const bool ok = (q < nbe) & (c < d.ncols);
        xv[u] = gj_load<T>(rx, ok ? (q + (c - c_lo) * d.ld) * (int)sizeof(T) : GJ_RSRC_RANGE);
    }
    // SC = old pivot columns with -I in the pivot rows; rows split over the
    // workgroups of this box (nobody writes those columns in this kernel).
    // Copied before the elimination, which does not need it: its loads
    // overlap the pivot block's and its stores drain during the elimination.
    // Unrolled so that eight independent loads are in flight per thread.
    const int nwg = (d.ncols + CHUNK - 1) / CHUNK;
    const int rows_per = (d.n + nwg - 1) / nwg;
    const int r0 = blockIdx.x * rows_per, r1 = min(d.n, r0 + rows_per);
    const int nr = max(0, r1 - r0);
    const int tot = nr * nbe;
    for (int e0 = 0; e0 < tot; e0 += 8 * 256) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256 + t;
            const int q2 = e / max(nr, 1), i = r0 + (e - q2 * nr);
            v[u] = (e < tot && !(i >= j0 && i < j0 + nbe)) ? d.X[i + (int64_t)(pc0 + q2) * d.ld] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256 + t;
            if (e < tot) {
                const int q2 = e / nr, i = r0 + (e - q2 * nr);
                const T w = (i >= j0 && i < j0 + nbe) ? ((i - j0 == q2) ? T(-1) : T(0)) : v[u];
                d.SC[i + (int64_t)q2 * d.n] = w;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ri + a, j = cj + b;
            if (!((i < nbe) & (j < nbe))) p[a][b] = i == j ? T(1) : T(0);
        }
#pragma unroll
    for (int u = 0; u < GJ_NB * CHUNK / 256; ++u) {
        const int e = t + 256 * u;
        Xp[e & (GJ_NB - 1)][e / GJ_NB] = xv[u];
    }
    if (t == 0) bad = 0;
    // Steps up to nbe rounded up to four run (past nbe the block is the
    // identity, which they leave unchanged); unrolled by four so that the
    // pivot's position inside a thread's 4 x 4 tile is a compile-time index
    // and only the ownership test is dynamic.
    const int nst = (nbe + 3) & ~3;
    if constexpr (!PAIR) {
        // publish row 0 and column 0
        if (ri == 0)
#pragma unroll
            for (int b = 0; b < 4; ++b) rowb[0][0][cj + b] = p[0][b];
        if (cj == 0)
#pragma unroll
            for (int a = 0; a < 4; ++a) colb[0][0][ri + a] = p[a][0];
        __syncthreads();
        for (int c4 = 0; c4 < nst; c4 += 4) {
            const bool own_r = ri == c4, own_c = cj == c4;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int c = c4 + l;
                const int buf = c & 1;
                const T piv = rowb[buf][0][c];
                if (t == 0 && !(fabs((double)piv) > 1e-300 && isfinite((double)piv))) bad = 1;
                const T inv = recip(piv);
                T prs[4], pcv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) prs[b] = rowb[buf][0][cj + b] * inv;
#pragma unroll
                for (int a = 0; a < 4; ++a) pcv[a] = colb[buf][0][ri + a];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) p[a][b] -= pcv[a] * prs[b];
                if (own_c)
#pragma unroll
                    for (int a = 0; a < 4; ++a) p[a][l] = -pcv[a] * inv;
                if (own_r)
#pragma unroll
                    for (int b = 0; b < 4; ++b) p[l][b] = prs[b];
                if (own_r && own_c) p[l][l] = inv;
                // publish row and column c + 1
                const int c1 = c + 1, nb2 = buf ^ 1;
                if (c1 < GJ_NB) {
                    const int l1 = (l + 1) & 3;
                    const bool r1 = ri == (c1 & ~3), k1 = cj == (c1 & ~3);
                    if (r1)
#pragma unroll
                        for (int b = 0; b < 4; ++b) rowb[nb2][0][cj + b] = p[l1][b];
                    if (k1)
#pragma unroll
                        for (int a = 0; a < 4; ++a) colb[nb2][0][ri + a] = p[a][l1];
                }
                __syncthreads();
            }
        }
    } else {
        // publish rows 0, 1 and columns 0, 1
        if (ri == 0)
#pragma unroll
            for (int b = 0; b < 4; ++b) { rowb[0][0][cj + b] = p[0][b]; rowb[0][1][cj + b] = p[1][b]; }
        if (cj == 0)
#pragma unroll
            for (int a = 0; a < 4; ++a) { colb[0][0][ri + a] = p[a][0]; colb[0][1][ri + a] = p[a][1]; }
        __syncthreads();
        for (int c4 = 0; c4 < nst; c4 += 4) {
            const bool own_r = ri == c4, own_c = cj == c4;
#pragma unroll
            for (int l = 0; l < 4; l += 2) {
                const int c = c4 + l;
                const int buf = (c >> 1) & 1;
                // 2 x 2 pivot block and its inverse
                const T b00 = rowb[buf][0][c], b01 = rowb[buf][0][c + 1];
                const T b10 = rowb[buf][1][c], b11 = rowb[buf][1][c + 1];
                const T det = b00 * b11 - b01 * b10;
                if (t == 0 && !(fabs((double)det) > 1e-300 && isfinite((double)det))) bad = 1;
                const T id = T(1) / det;
                const T i00 = b11 * id, i01 = -b01 * id, i10 = -b10 * id, i11 = b00 * id;
                // the pivot rows times the inverse, and the old pivot columns
                T r0[4], r1[4], c0[4], c1v[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T x0 = rowb[buf][0][cj + b], x1 = rowb[buf][1][cj + b];
                    r0[b] = i00 * x0 + i01 * x1;
                    r1[b] = i10 * x0 + i11 * x1;
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) { c0[a] = colb[buf][0][ri + a]; c1v[a] = colb[buf][1][ri + a]; }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) p[a][b] -= c0[a] * r0[b] + c1v[a] * r1[b];
                if (own_c)
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        p[a][l] = -(c0[a] * i00 + c1v[a] * i10);
                        p[a][l + 1] = -(c0[a] * i01 + c1v[a] * i11);
                    }
                if (own_r)
#pragma unroll
                    for (int b = 0; b < 4; ++b) { p[l][b] = r0[b]; p[l + 1][b] = r1[b]; }
                if (own_r && own_c) {
                    p[l][l] = i00; p[l][l + 1] = i01;
                    p[l + 1][l] = i10; p[l + 1][l + 1] = i11;
                }
                // publish rows and columns c + 2, c + 3
                const int c2 = c + 2, nb2 = buf ^ 1;
                if (c2 < GJ_NB) {
                    const int l2 = (l + 2) & 3;
                    const bool rr = ri == (c2 & ~3), kk = cj == (c2 & ~3);
                    if (rr)
#pragma unroll
                        for (int b = 0; b < 4; ++b) { rowb[nb2][0][cj + b] = p[l2][b]; rowb[nb2][1][cj + b] = p[l2 + 1][b]; }
                    if (kk)
#pragma unroll
                        for (int a = 0; a < 4; ++a) { colb[nb2][0][ri + a] = p[a][l2]; colb[nb2][1][ri + a] = p[a][l2 + 1]; }
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) Pi[ri + a][cj + b] = p[a][b];
    __syncthreads();
    if (t == 0 && bad && blockIdx.x == 0) atomicCAS(d.err ? d.err : err, 0, d.box + 1);
    // SR = P^{-1} X[piv rows, chunk] on the matrix cores: wave w owns the
    // 32 x 32 block (rows 32 (w / 2), columns 32 (w % 2)) as 2 x 2 MFMA blocks
    // over K = 64.  The MFMA computes the transposed block, so lane l holds
    // rows q0 + l % 16 of SR (contiguous in memory) and the stores coalesce.
    // Entries past nbe are zero in X and identity in P, so K runs to 64.
    {
        const int lane = t & 63, wave = t >> 6;
        typename GjMfma<T>::acc_t acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = typename GjMfma<T>::acc_t{0, 0, 0, 0};
        const int qw = 32 * (wave >> 1), cw = 32 * (wave & 1);
#pragma unroll 4
        for (int kk = 0; kk < GJ_NB; kk += 4) {
            const int k = kk + (lane >> 4);
            T a[2], b[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) a[bi] = Pi[qw + 16 * bi + (lane & 15)][k];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) b[bj] = Xp[k][cw + 16 * bj + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = GjMfma<T>::step(b[bj], a[bi], acc[bi][bj]);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = qw + 16 * bi + (lane & 15);
                    const int c = c_lo + cw + 16 * bj + GjMfma<T>::col(lane, v);
                    if (q >= nbe || c >= d.ncols) continue;
                    const bool pivc = c >= pc0 && c < pc0 + nbe;
                    d.SR[q + (int64_t)c * nb] = pivc ? Pi[q][c - pc0] : acc[bi][bj][v];
                    if (!pivc) d.X[(j0 + q) + (int64_t)c * d.ld] = T(0);
                }
    }
}

}  // namespace

template <typename T>
void launch_gj_pivot(const GJDesc<T>* d, int n_desc, int step, int nb, int max_chunks, int* err,
                     int pair, hipStream_t s) {
    constexpr int MAX_Y = 65535;   // grid y limit: blocks beyond it go to further launches
    for (int o = 0; o < n_desc; o += MAX_Y) {
        const dim3 grid(max_chunks, std::min(MAX_Y, n_desc - o));
        if (pair)
            hipLaunchKernelGGL((gj_pivot_kernel<T, true>), grid, dim3(256), 0, s, d + o, step, nb, err);
        else
            hipLaunchKernelGGL((gj_pivot_kernel<T, false>), grid, dim3(256), 0, s, d + o, step, nb, err);
    }
}

template void launch_gj_pivot<double>(const GJDesc<double>*, int, int, int, int, int*, int, hipStream_t);
template void launch_gj_pivot<float>(const GJDesc<float>*, int, int, int, int, int*, int, hipStream_t);

}  // namespace rsd
