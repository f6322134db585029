// Data movement of the inverse apply (Algorithm 6) between tree levels.
//
// Each box keeps its vector block in [skeleton; residual] order.  The
// upward pass hands a box's reduced right-hand side g (length k) to its
// parent, where the two children's skeletons form the parent's active set;
// the downward pass hands the parent's solution on those points back.  The
// maps are the layouts' inverse position tables, shared by every box of a
// type.  Leaves read the caller's right-hand side through the grid
// permutation and write the solution back through it.
#include "common.hpp"

namespace rsd {

namespace {

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) gather_leaf_kernel(
    TD* __restrict__ V, const TS* __restrict__ f, int64_t ldf, int nrhs,
    const BoxDev* __restrict__ boxes, const int* __restrict__ box_ids,
    const LayoutDev* __restrict__ layouts, const int* __restrict__ lu, const int* __restrict__ lv,
    const int64_t* __restrict__ perm, int64_t ny, int64_t plane_off) {
    const BoxDev b = boxes[box_ids[blockIdx.y]];
    const LayoutDev L = layouts[b.layout];
    const int m = L.k + L.r;
    TD* Vb = V + b.offV * nrhs;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < m * nrhs; e += gridDim.x * 256) {
        const int q = e % m, c = e / m;
        int64_t g = (int64_t)(b.x0 + lu[L.off_uv + q]) * ny + (b.y0 + lv[L.off_uv + q]);
        if (plane_off) g += dof_plane(q, L.k, L.r) * plane_off;
        Vb[q + (int64_t)c * m] = (TD)f[perm[g] + c * ldf];
    }
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) scatter_leaf_kernel(
    TD* __restrict__ x, int64_t ldx, const TS* __restrict__ V, const TS* __restrict__ Y, int nrhs,
    const BoxDev* __restrict__ boxes, const int* __restrict__ box_ids,
    const LayoutDev* __restrict__ layouts, const int* __restrict__ lu, const int* __restrict__ lv,
    const int64_t* __restrict__ perm, int64_t ny, int64_t plane_off) {
    const BoxDev b = boxes[box_ids[blockIdx.y]];
    const LayoutDev L = layouts[b.layout];
    const int m = L.k + L.r;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < m * nrhs; e += gridDim.x * 256) {
        const int q = e % m, c = e / m;
        int64_t g = (int64_t)(b.x0 + lu[L.off_uv + q]) * ny + (b.y0 + lv[L.off_uv + q]);
        if (plane_off) g += dof_plane(q, L.k, L.r) * plane_off;
        const TS v = q < L.k ? V[b.offV * nrhs + q + (int64_t)c * m]
                             : Y[b.offY * nrhs + (q - L.k) + (int64_t)c * L.r];
        x[perm[g] + c * ldx] = (TD)v;
    }
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) scatter_up_kernel(
    TD* __restrict__ Vp, const TS* __restrict__ V, int nrhs, const BoxDev* __restrict__ boxes,
    const int* __restrict__ box_ids, const LayoutDev* __restrict__ layouts,
    const int* __restrict__ inv) {
    const BoxDev b = boxes[box_ids[blockIdx.y]];
    const BoxDev P = boxes[b.parent];
    const LayoutDev LP = layouts[P.layout];
    const int m = b.k + b.r, mp = P.k + P.r;
    const int* map = inv + (b.pos == 0 ? LP.off_inv0 : LP.off_inv1);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < b.k * nrhs; e += gridDim.x * 256) {
        const int i = e % b.k, c = e / b.k;
        Vp[P.offV * nrhs + map[i] + (int64_t)c * mp] = (TD)V[b.offV * nrhs + i + (int64_t)c * m];
    }
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) gather_down_kernel(
    TD* __restrict__ V, const TS* __restrict__ Vp, const TS* __restrict__ Yp, int nrhs,
    const BoxDev* __restrict__ boxes, const int* __restrict__ box_ids,
    const LayoutDev* __restrict__ layouts, const int* __restrict__ inv) {
    const BoxDev b = boxes[box_ids[blockIdx.y]];
    const BoxDev P = boxes[b.parent];
    const LayoutDev LP = layouts[P.layout];
    const int m = b.k + b.r, mp = P.k + P.r;
    const int* map = inv + (b.pos == 0 ? LP.off_inv0 : LP.off_inv1);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < b.k * nrhs; e += gridDim.x * 256) {
        const int i = e % b.k, c = e / b.k;
        const int q = map[i];
        const TS v = q < P.k ? Vp[P.offV * nrhs + q + (int64_t)c * mp]
                             : Yp[P.offY * nrhs + (q - P.k) + (int64_t)c * P.r];
        V[b.offV * nrhs + i + (int64_t)c * m] = (TD)v;
    }
}

inline int chunks(int64_t n) {
    int64_t c = (n + 1023) / 1024;
    return (int)(c < 1 ? 1 : (c > 2048 ? 2048 : c));
}

template <typename TS, typename TD>
__global__ void convert_kernel(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        d[i] = (TD)s[i];
}

// to_grid: dst[g + c*N] = src[perm[g]*width.. ] ; else dst[perm[g]] = src[g]
__global__ void permute_kernel(double* __restrict__ dst, const double* __restrict__ src,
                               const int64_t* __restrict__ perm, int64_t n, int nrhs, int width,
                               int to_grid) {
    const int64_t tot = n * nrhs * width;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int w = (int)(e % width);
        const int64_t g = (e / width) % n;
        const int64_t c = e / (width * n);
        const int64_t p = perm[g];
        if (to_grid) dst[(g + c * n) * width + w] = src[(p + c * n) * width + w];
        else dst[(p + c * n) * width + w] = src[(g + c * n) * width + w];
    }
}

__global__ void resid_kernel(double* __restrict__ r, const double* __restrict__ f,
                             const double* __restrict__ ax, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        r[i] = f[i] - ax[i];
}

__global__ void add_kernel(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x[i] += d[i];
}

// out[c] = sum_i x[i + c*n]^2, one workgroup per column (fixed reduction order)
// Squared column norms in two passes with a fixed summation order (the
// refinement's convergence test gives the same decision on every run):
// pass 1, COLNORM_PARTS workgroups per column, each a contiguous part;
// pass 2, one workgroup per column adds the parts.
constexpr int COLNORM_PARTS = COLNORM_WS_PER_COL;
static_assert(COLNORM_PARTS <= 256, "one partial per thread of the summing workgroup");

__device__ inline double block_sum256(double s, double* red) {
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(256) colnorm_part_kernel(double* __restrict__ part,
                                                           const double* __restrict__ x, int64_t n) {
    __shared__ double red[256];
    const double* col = x + blockIdx.y * n;
    const int64_t len = (n + COLNORM_PARTS - 1) / COLNORM_PARTS;
    const int64_t i0 = blockIdx.x * len, i1 = min(n, i0 + len);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += col[i] * col[i];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) part[blockIdx.y * COLNORM_PARTS + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) colnorm_sum_kernel(double* __restrict__ out,
                                                          const double* __restrict__ part) {
    __shared__ double red[256];
    const double s = threadIdx.x < COLNORM_PARTS ? part[blockIdx.x * COLNORM_PARTS + threadIdx.x] : 0.0;
    const double t = block_sum256(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// Right-hand side of the factored system from a grid-ordered one (N x nrhs,
// float64, or interleaved complex when cplx): scaled by 1/sqrt(b) (sb given;
// the contrast form A = S M S, S = diag sqrt b) and, for complex vectors,
// split into the two dof planes of J: R = [Re; Im] per column (ld 2N).
__global__ void scale_split_kernel(double* __restrict__ R, const double* __restrict__ f,
                                   const double* __restrict__ sb, int64_t N, int nrhs, int cplx) {
    const int64_t tot = N * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t g = e % N, c = e / N;
        const double s = sb ? 1.0 / sb[g] : 1.0;
        if (cplx) {
            R[g + c * 2 * N] = s * f[2 * e];
            R[N + g + c * 2 * N] = s * f[2 * e + 1];
        } else {
            R[e] = s * f[e];
        }
    }
}

// Inverse of the above for the solution: x = S^-1 (u - i w) (complex) or
// S^-1 u, from the dof planes [u; w] of J.
__global__ void scale_merge_kernel(double* __restrict__ x, const double* __restrict__ X,
                                   const double* __restrict__ sb, int64_t N, int nrhs, int cplx) {
    const int64_t tot = N * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t g = e % N, c = e / N;
        const double s = sb ? 1.0 / sb[g] : 1.0;
        if (cplx) {
            x[2 * e] = s * X[g + c * 2 * N];
            x[2 * e + 1] = -s * X[N + g + c * 2 * N];
        } else {
            x[e] = s * X[e];
        }
    }
}

__global__ void finite_kernel(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        if (!isfinite(x[i])) atomicOr(flag, 1);
}

}  // namespace

template <typename TS, typename TD>
void launch_gather_leaf(TD* V, const TS* f, int64_t ldf, int nrhs, const BoxDev* boxes,
                        const int* box_ids, int n_boxes, const LayoutDev* layouts, const int* lu,
                        const int* lv, const int64_t* perm, int64_t ny, int64_t plane_off, int max_m,
                        hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL((gather_leaf_kernel<TS, TD>), dim3(chunks((int64_t)max_m * nrhs), n_boxes),
                       dim3(256), 0, s, V, f, ldf, nrhs, boxes, box_ids, layouts, lu, lv, perm, ny,
                       plane_off);
}
template <typename TS, typename TD>
void launch_scatter_leaf(TD* x, int64_t ldx, const TS* V, const TS* Y, int nrhs,
                         const BoxDev* boxes, const int* box_ids, int n_boxes,
                         const LayoutDev* layouts, const int* lu, const int* lv,
                         const int64_t* perm, int64_t ny, int64_t plane_off, int max_m, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL((scatter_leaf_kernel<TS, TD>), dim3(chunks((int64_t)max_m * nrhs), n_boxes),
                       dim3(256), 0, s, x, ldx, V, Y, nrhs, boxes, box_ids, layouts, lu, lv, perm, ny,
                       plane_off);
}
template <typename TS, typename TD>
void launch_scatter_up(TD* Vparent, const TS* V, int nrhs, const BoxDev* boxes, const int* box_ids,
                       int n_boxes, const LayoutDev* layouts, const int* inv, int max_k,
                       hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL((scatter_up_kernel<TS, TD>), dim3(chunks((int64_t)max_k * nrhs), n_boxes),
                       dim3(256), 0, s, Vparent, V, nrhs, boxes, box_ids, layouts, inv);
}
template <typename TS, typename TD>
void launch_gather_down(TD* V, const TS* Vparent, const TS* Yparent, int nrhs,
                        const BoxDev* boxes, const int* box_ids, int n_boxes,
                        const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL((gather_down_kernel<TS, TD>), dim3(chunks((int64_t)max_k * nrhs), n_boxes),
                       dim3(256), 0, s, V, Vparent, Yparent, nrhs, boxes, box_ids, layouts, inv);
}
template <typename TS, typename TD>
void launch_convert(TD* dst, const TS* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((convert_kernel<TS, TD>), dim3(chunks(n)), dim3(256), 0, s, dst, src, n);
}
void launch_permute(double* dst, const double* src, const int64_t* perm, int64_t n, int nrhs,
                    int width, int to_grid, hipStream_t s) {
    hipLaunchKernelGGL(permute_kernel, dim3(chunks(n * nrhs * width)), dim3(256), 0, s, dst, src,
                       perm, n, nrhs, width, to_grid);
}
void launch_axpy_resid(double* r, const double* f, const double* Ax, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(resid_kernel, dim3(chunks(n)), dim3(256), 0, s, r, f, Ax, n);
}
void launch_add(double* x, const double* d, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(add_kernel, dim3(chunks(n)), dim3(256), 0, s, x, d, n);
}
void launch_col_norms2(double* out, const double* x, int64_t n, int ncols, double* ws, hipStream_t s) {
    if (ncols <= 0) return;
    hipLaunchKernelGGL(colnorm_part_kernel, dim3(COLNORM_PARTS, ncols), dim3(256), 0, s, ws, x, n);
    hipLaunchKernelGGL(colnorm_sum_kernel, dim3(ncols), dim3(256), 0, s, out, ws);
}
void launch_scale_split(double* R, const double* f, const double* sb, int64_t N, int nrhs, int cplx,
                        hipStream_t s) {
    hipLaunchKernelGGL(scale_split_kernel, dim3(chunks(N * nrhs)), dim3(256), 0, s, R, f, sb, N, nrhs, cplx);
}
void launch_scale_merge(double* x, const double* X, const double* sb, int64_t N, int nrhs, int cplx,
                        hipStream_t s) {
    hipLaunchKernelGGL(scale_merge_kernel, dim3(chunks(N * nrhs)), dim3(256), 0, s, x, X, sb, N, nrhs, cplx);
}
void launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(finite_kernel, dim3(chunks(n)), dim3(256), 0, s, x, n, flag);
}

#define INST2(TS, TD)                                                                              \
    template void launch_gather_leaf<TS, TD>(TD*, const TS*, int64_t, int, const BoxDev*,          \
                                             const int*, int, const LayoutDev*, const int*,        \
                                             const int*, const int64_t*, int64_t, int64_t, int,    \
                                             hipStream_t);                                         \
    template void launch_scatter_leaf<TD, TS>(TS*, int64_t, const TD*, const TD*, int,             \
                                              const BoxDev*, const int*, int, const LayoutDev*,    \
                                              const int*, const int*, const int64_t*, int64_t,     \
                                              int64_t, int, hipStream_t);                          \
    template void launch_convert<TS, TD>(TD*, const TS*, int64_t, hipStream_t);
INST2(double, double)
INST2(double, float)
INST2(float, double)
#undef INST2
#define INST3(TS, TD)                                                                              \
    template void launch_scatter_up<TS, TD>(TD*, const TS*, int, const BoxDev*, const int*, int,   \
                                            const LayoutDev*, const int*, int, hipStream_t);       \
    template void launch_gather_down<TS, TD>(TD*, const TS*, const TS*, int, const BoxDev*,        \
                                             const int*, int, const LayoutDev*, const int*, int,   \
                                             hipStream_t);
INST3(double, double)
INST3(float, float)
INST3(float, double)
INST3(double, float)
#undef INST3

}  // namespace rsd
