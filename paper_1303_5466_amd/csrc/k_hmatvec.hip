// Compressed forward product y ~ A x through the factor's own skeletonization
// (Sec. 2.3: the matrix itself in the recursive-skeleton form, O(N) work).
//
// The block of A between two distinct boxes i, j is L_i A(sk_i, sk_j) R_j, so
// A = D + L A~ R telescopes up the tree (R_b = [I T_b] on a box's [sk; rs]
// active vector, L_b = R_b^T):
//   up      skeleton charges x^_b = x_b[sk] + T_b x_b[rs], written into the
//           parent's active vector (the children's skeletons);
//   across  every box above the leaves adds to each child's skeleton
//           potential the kernel block to its sibling's skeleton times the
//           sibling's charges (kernel values evaluated on the fly);
//   down    a box's potential spreads to its active points, [p; T_b^T p],
//           and on into its children's potentials;
//   leaves  the spread plus the box's own dense block A(I_i, I_i) x_i.
// Vectors per box in the solve's layout (offV, k + r entries per right-hand
// side, column-major over the right-hand sides), float64 throughout; as in
// the solve, the boxes of float32 and float64 levels number their offsets
// separately, so every kernel takes the base of each level it touches.
// Laplace kernel; T is read in the precision its level keeps.
#include "common.hpp"

namespace rsd {

namespace {

constexpr double H_INV_2PI = 0.15915494309189533576888376337251;

// A between two distinct points at grid offsets (du, dv): h^2 (1/2pi) log r
__device__ inline double lap_off(const KernelDesc& kd, int du, int dv) {
    return kd.h * kd.h * H_INV_2PI * (kd.logh + 0.5 * log((double)(du * du + dv * dv)));
}

// up: x^ of every box of a level into its parent's active vector
template <typename TT>
__global__ void __launch_bounds__(256) hmv_up_kernel(const double* __restrict__ X, double* __restrict__ Xpar,
                                                      const TT* __restrict__ Tarena,
                                                      int nrhs, const BoxDev* __restrict__ boxes,
                                                      const int* __restrict__ ids,
                                                      const LayoutDev* __restrict__ layouts,
                                                      const int* __restrict__ inv) {
    const BoxDev b = boxes[ids[blockIdx.y]];
    const LayoutDev L = layouts[b.layout];
    const BoxDev P = boxes[b.parent];
    const LayoutDev LP = layouts[P.layout];
    const int m = b.k + b.r, mp = P.k + P.r;
    const int* map = inv + (b.pos == 0 ? LP.off_inv0 : LP.off_inv1);
    const double* Xb = X + b.offV * nrhs;
    const TT* T = L.offT >= 0 ? Tarena + L.offT : nullptr;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < b.k * nrhs; e += gridDim.x * 256) {
        const int i = e % b.k, c = e / b.k;
        const double* xc = Xb + (int64_t)c * m;
        double s = xc[i];
        if (T)
            for (int j = 0; j < b.r; ++j) s += (double)T[i + (int64_t)j * b.k] * xc[b.k + j];
        Xpar[P.offV * nrhs + map[i] + (int64_t)c * mp] = s;
    }
}

// across: for every parent, the rows of both children's skeleton potentials
// (blockIdx.x * 256 + thread over the k1 + k2 rows and the right-hand sides)
__global__ void __launch_bounds__(256) hmv_sibling_kernel(double* __restrict__ Pot, const double* __restrict__ Xpar,
                                                          int nrhs, const BoxDev* __restrict__ boxes,
                                                          const int* __restrict__ ids,
                                                          const LayoutDev* __restrict__ layouts,
                                                          const int* __restrict__ lu, const int* __restrict__ lv,
                                                          const int* __restrict__ inv, KernelDesc kd) {
    const BoxDev P = boxes[ids[blockIdx.y]];
    const LayoutDev LP = layouts[P.layout];
    const BoxDev C0 = boxes[P.child0], C1 = boxes[P.child1];
    const LayoutDev L0 = layouts[C0.layout], L1 = layouts[C1.layout];
    const int k0 = C0.k, k1 = C1.k, mp = P.k + P.r;
    const double* Xp = Xpar + P.offV * nrhs;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < (k0 + k1) * nrhs; e += gridDim.x * 256) {
        const int row = e % (k0 + k1), c = e / (k0 + k1);
        // the receiving child (own) and its sibling (other)
        const bool first = row < k0;
        const BoxDev& own = first ? C0 : C1;
        const BoxDev& oth = first ? C1 : C0;
        const LayoutDev& Lo = first ? L0 : L1;
        const LayoutDev& Ls = first ? L1 : L0;
        const int i = first ? row : row - k0;
        const int ks = first ? k1 : k0;
        const int* smap = inv + (first ? LP.off_inv1 : LP.off_inv0);   // sibling's charges in the parent
        const int gu = own.x0 + lu[Lo.off_uv + i], gv = own.y0 + lv[Lo.off_uv + i];
        double s = 0.0;
        for (int j = 0; j < ks; ++j) {
            const int du = gu - (oth.x0 + lu[Ls.off_uv + j]), dv = gv - (oth.y0 + lv[Ls.off_uv + j]);
            s += lap_off(kd, du, dv) * Xp[smap[j] + (int64_t)c * mp];
        }
        Pot[own.offV * nrhs + i + (int64_t)c * (own.k + own.r)] += s;
    }
}

// down: a box's potential on its active points, [p; T^T p], kept in Y
template <typename TT>
__global__ void __launch_bounds__(256) hmv_spread_kernel(double* __restrict__ Y, const double* __restrict__ Pot,
                                                          const TT* __restrict__ Tarena, int nrhs,
                                                          const BoxDev* __restrict__ boxes,
                                                          const int* __restrict__ ids,
                                                          const LayoutDev* __restrict__ layouts) {
    const BoxDev b = boxes[ids[blockIdx.y]];
    const LayoutDev L = layouts[b.layout];
    const int m = b.k + b.r;
    const TT* T = L.offT >= 0 ? Tarena + L.offT : nullptr;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < m * nrhs; e += gridDim.x * 256) {
        const int q = e % m, c = e / m;
        const double* pc = Pot + b.offV * nrhs + (int64_t)c * m;
        double s = 0.0;
        if (q < b.k) s = pc[q];
        else if (T)
            for (int i = 0; i < b.k; ++i) s += (double)T[i + (int64_t)(q - b.k) * b.k] * pc[i];
        Y[b.offV * nrhs + q + (int64_t)c * m] = s;
    }
}

// down: each child's potential takes its part of the parent's spread
__global__ void __launch_bounds__(256) hmv_push_kernel(double* __restrict__ Pot, const double* __restrict__ Ypar,
                                                       int nrhs, const BoxDev* __restrict__ boxes,
                                                       const int* __restrict__ ids,
                                                       const LayoutDev* __restrict__ layouts,
                                                       const int* __restrict__ inv) {
    const BoxDev b = boxes[ids[blockIdx.y]];
    const BoxDev P = boxes[b.parent];
    const LayoutDev LP = layouts[P.layout];
    const int m = b.k + b.r, mp = P.k + P.r;
    const int* map = inv + (b.pos == 0 ? LP.off_inv0 : LP.off_inv1);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < b.k * nrhs; e += gridDim.x * 256) {
        const int i = e % b.k, c = e / b.k;
        Pot[b.offV * nrhs + i + (int64_t)c * m] += Ypar[P.offV * nrhs + map[i] + (int64_t)c * mp];
    }
}

// leaves: the spread potential plus the dense leaf block times the leaf's x,
// written to the caller's order through the grid permutation
template <typename TT>
__global__ void __launch_bounds__(256) hmv_leaf_kernel(double* __restrict__ y, int64_t ldy,
                                                        const double* __restrict__ X,
                                                        const double* __restrict__ Pot,
                                                        const TT* __restrict__ Tarena, int nrhs,
                                                        const BoxDev* __restrict__ boxes,
                                                        const int* __restrict__ ids,
                                                        const LayoutDev* __restrict__ layouts,
                                                        const int* __restrict__ lu, const int* __restrict__ lv,
                                                        const int64_t* __restrict__ perm, KernelDesc kd) {
    const BoxDev b = boxes[ids[blockIdx.y]];
    const LayoutDev L = layouts[b.layout];
    const int m = b.k + b.r;
    const TT* T = L.offT >= 0 ? Tarena + L.offT : nullptr;
    const bool has_pot = b.parent >= 0;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < m * nrhs; e += gridDim.x * 256) {
        const int q = e % m, c = e / m;
        const double* xc = X + b.offV * nrhs + (int64_t)c * m;
        const int uq = lu[L.off_uv + q], vq = lv[L.off_uv + q];
        const int64_t g = (int64_t)(b.x0 + uq) * kd.ny + (b.y0 + vq);
        double s = 0.0;
        if (has_pot) {
            const double* pc = Pot + b.offV * nrhs + (int64_t)c * m;
            if (q < b.k) s = pc[q];
            else if (T)
                for (int i = 0; i < b.k; ++i) s += (double)T[i + (int64_t)(q - b.k) * b.k] * pc[i];
        }
        for (int j = 0; j < m; ++j) {
            const double a = j == q ? (kd.a ? kd.a[g] : 1.0) + kd.sc_re
                                    : lap_off(kd, uq - lu[L.off_uv + j], vq - lv[L.off_uv + j]);
            s += a * xc[j];
        }
        y[perm[g] + (int64_t)c * ldy] = s;
    }
}

inline dim3 grid_for(int64_t work, int n_boxes) {
    int64_t c = (work + 255) / 256;
    if (c < 1) c = 1;
    if (c > 1024) c = 1024;
    return dim3((unsigned)c, (unsigned)n_boxes);
}

}  // namespace

template <typename TT>
void launch_hmv_up(const double* X, double* Xpar, const TT* Tarena, int nrhs, const BoxDev* boxes, const int* ids,
                   int n_boxes, const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL(hmv_up_kernel<TT>, grid_for((int64_t)max_k * nrhs, n_boxes), dim3(256), 0, s, X, Xpar,
                       Tarena, nrhs, boxes, ids, layouts, inv);
}

void launch_hmv_sibling(double* Pot, const double* Xpar, int nrhs, const BoxDev* boxes, const int* ids, int n_boxes,
                        const LayoutDev* layouts, const int* lu, const int* lv, const int* inv, int max_kk,
                        const KernelDesc& kd, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL(hmv_sibling_kernel, grid_for((int64_t)max_kk * nrhs, n_boxes), dim3(256), 0, s, Pot, Xpar,
                       nrhs, boxes, ids, layouts, lu, lv, inv, kd);
}

template <typename TT>
void launch_hmv_spread(double* Y, const double* Pot, const TT* Tarena, int nrhs, const BoxDev* boxes,
                       const int* ids, int n_boxes, const LayoutDev* layouts, int max_m, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL(hmv_spread_kernel<TT>, grid_for((int64_t)max_m * nrhs, n_boxes), dim3(256), 0, s, Y, Pot,
                       Tarena, nrhs, boxes, ids, layouts);
}

void launch_hmv_push(double* Pot, const double* Ypar, int nrhs, const BoxDev* boxes, const int* ids, int n_boxes,
                     const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL(hmv_push_kernel, grid_for((int64_t)max_k * nrhs, n_boxes), dim3(256), 0, s, Pot, Ypar, nrhs,
                       boxes, ids, layouts, inv);
}

template <typename TT>
void launch_hmv_leaf(double* y, int64_t ldy, const double* X, const double* Pot, const TT* Tarena, int nrhs,
                     const BoxDev* boxes, const int* ids, int n_boxes, const LayoutDev* layouts, const int* lu,
                     const int* lv, const int64_t* perm, int max_m, const KernelDesc& kd, hipStream_t s) {
    if (n_boxes <= 0) return;
    hipLaunchKernelGGL(hmv_leaf_kernel<TT>, grid_for((int64_t)max_m * nrhs, n_boxes), dim3(256), 0, s, y, ldy, X,
                       Pot, Tarena, nrhs, boxes, ids, layouts, lu, lv, perm, kd);
}

#define INST(TT)                                                                                       \
    template void launch_hmv_up<TT>(const double*, double*, const TT*, int, const BoxDev*, const int*, \
                                    int, const LayoutDev*, const int*, int, hipStream_t);              \
    template void launch_hmv_spread<TT>(double*, const double*, const TT*, int, const BoxDev*,         \
                                        const int*, int, const LayoutDev*, int, hipStream_t);          \
    template void launch_hmv_leaf<TT>(double*, int64_t, const double*, const double*, const TT*, int,  \
                                      const BoxDev*, const int*, int, const LayoutDev*, const int*,    \
                                      const int*, const int64_t*, int, const KernelDesc&, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace rsd
