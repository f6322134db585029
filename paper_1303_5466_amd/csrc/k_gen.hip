// Kernel-matrix generation from grid coordinates (Sec. 5, general
// formulation; the Helmholtz kernel of Sec. 5.3 on two dofs per point, see
// KernelDesc): leaf diagonal blocks D_i, the parent blocks
// F_i = D_i + diag(E_c1, E_c2) of Algorithm 1 (sibling interactions
// generated on the fly, children's E_c gathered), and the proxy matrices
// [K(Z, X^sk) | K(Z, X^rs)] of the interpolation problem (Sec. 3.1).
//
// All coordinates are integer grid offsets relative to a box origin; the
// kernel depends on the distance only, so K(h |(du, dv)|) is evaluated from
// du^2 + dv^2 directly.  Writes are column-major and coalesced (consecutive
// threads take consecutive rows).
#include "common.hpp"

namespace rsd {

namespace {

// Walk over the elements e = i + j * rows of a column-major block, from e0 in
// steps of `stride`: the row and column are carried from step to step, so the
// loop needs no 64-bit division per element (only the first position is
// divided out).  rows > 0.
struct ColWalk {
    int64_t e;
    int i, j, di, dj, rows;
    __device__ ColWalk(int64_t e0, int64_t stride, int rows_) : e(e0), rows(rows_) {
        i = (int)(e0 % rows_);
        j = (int)(e0 / rows_);
        di = (int)(stride % rows_);
        dj = (int)(stride / rows_);
    }
    __device__ void next(int64_t stride) {
        e += stride;
        i += di;
        j += dj;
        if (i >= rows) {
            i -= rows;
            ++j;
        }
    }
};


constexpr double INV_2PI = 0.15915494309189533576888376337251;

// K(h * sqrt(rho2)) for rho2 > 0 (Laplace: (1/2pi) log r)
__device__ inline double kernel_val(const KernelDesc& kd, double rho2) {
    return INV_2PI * (kd.logh + 0.5 * log(rho2));
}
__device__ inline float kernel_val_f(const KernelDesc& kd, float rho2) {
    return (float)INV_2PI * ((float)kd.logh + 0.5f * logf(rho2));
}

template <typename T> struct KV;
template <> struct KV<double> {
    __device__ static double off(const KernelDesc& kd, int du, int dv) {
        return kd.h * kd.h * kernel_val(kd, (double)(du * du + dv * dv));
    }
    __device__ static double proxy(const KernelDesc& kd, int du, int dv) {
        return kernel_val(kd, (double)(du * du + dv * dv));
    }
};
template <> struct KV<float> {
    __device__ static float off(const KernelDesc& kd, int du, int dv) {
        return (float)(kd.h * kd.h) * kernel_val_f(kd, (float)(du * du + dv * dv));
    }
    __device__ static float proxy(const KernelDesc& kd, int du, int dv) {
        return kernel_val_f(kd, (float)(du * du + dv * dv));
    }
};

template <typename T>
__device__ inline T diag_val(const KernelDesc& kd, int64_t g) {
    if (kd.has_b) return T(1.0 + kd.sb[g] * kd.sb[g] * kd.sc_re);
    return T((kd.a ? kd.a[g] : 1.0) + kd.sc_re);
}

// Helmholtz G(r) = (i/4) H0^(1)(k r) = -Y0(k r)/4 + i J0(k r)/4 at r = h sqrt(rho2)
__device__ inline void helmholtz_val(const KernelDesc& kd, double rho2, double& gr, double& gi) {
    const double z = kd.k * kd.h * sqrt(rho2);
    gr = -0.25 * y0(z);
    gi = 0.25 * j0(z);
}

// Complex factors: the (pi, pj) component of J of the entry between two dofs
// of points at offsets (du, dv) (same point: du = dv = 0, grid index g) --
// a_g + sc on the diagonal, h^2 G off it (scale = h^2), or the proxy kernel
// G itself (scale = 1).
__device__ inline double cplx_entry(const KernelDesc& kd, int du, int dv, int64_t g, int pi, int pj,
                                    double scale) {
    if (du == 0 && dv == 0) return jform((kd.a ? kd.a[g] : 1.0) + kd.sc_re, kd.sc_im, pi, pj);
    double gr, gi;
    helmholtz_val(kd, (double)(du * du + dv * dv), gr, gi);
    return scale * jform(gr, gi, pi, pj);
}

// Leaf block D_i of one box: kernel entries off the diagonal, the
// identity coefficient plus the self-cell integral on it.
template <typename T, bool CPLX>
__device__ inline void leaf_F_box(T* __restrict__ F, const BoxDev* __restrict__ boxes, int box,
                                  const LayoutDev* __restrict__ layouts, const int* __restrict__ lu,
                                  const int* __restrict__ lv, const KernelDesc& kd) {
    const BoxDev b = boxes[box];
    const LayoutDev L = layouts[b.layout];
    const int m = L.k + L.r;
    T* Fb = F + b.offF;
    const int* U = lu + L.off_uv;
    const int* V = lv + L.off_uv;
    const int64_t stride_ = (int64_t)gridDim.x * 256;
    if ((int64_t)m * m > 0)
    for (ColWalk w(blockIdx.x * 256 + threadIdx.x, stride_, m); w.e < (int64_t)m * m; w.next(stride_)) {
        const int64_t e = w.e;
        const int i = w.i, j = w.j;
        if constexpr (CPLX) {
            const int64_t g = (int64_t)(b.x0 + U[i]) * kd.ny + (b.y0 + V[i]);
            Fb[e] = T(cplx_entry(kd, U[i] - U[j], V[i] - V[j], g, dof_plane(i, L.k, L.r),
                                 dof_plane(j, L.k, L.r), kd.h * kd.h));
            continue;
        }
        T val;
        if (i == j) {
            const int64_t g = (int64_t)(b.x0 + U[i]) * kd.ny + (b.y0 + V[i]);
            val = diag_val<T>(kd, g);
        } else {
            val = KV<T>::off(kd, U[i] - U[j], V[i] - V[j]);
            if (kd.has_b) {
                const int64_t gi = (int64_t)(b.x0 + U[i]) * kd.ny + (b.y0 + V[i]);
                const int64_t gj = (int64_t)(b.x0 + U[j]) * kd.ny + (b.y0 + V[j]);
                val = val * T(kd.sb[gi] * kd.sb[gj]);
            }
        }
        Fb[e] = val;
    }
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) leaf_F_kernel(T* __restrict__ F, const BoxDev* __restrict__ boxes,
                                                      const int* __restrict__ box_ids,
                                                      const LayoutDev* __restrict__ layouts,
                                                      const int* __restrict__ lu,
                                                      const int* __restrict__ lv, KernelDesc kd) {
    leaf_F_box<T, CPLX>(F, boxes, box_ids[blockIdx.y], layouts, lu, lv, kd);
}

// the boxes of several factors (a batch group): item y = (factor, box)
template <typename T>
__global__ void __launch_bounds__(256) leaf_F_group_kernel(const AsmInst* __restrict__ insts,
                                                            const GroupItem* __restrict__ items) {
    const GroupItem it = items[blockIdx.y];
    const AsmInst& I = insts[it.inst];
    leaf_F_box<T, false>(static_cast<T*>(I.F), I.boxes, it.box, I.layouts, I.lu, I.lv, I.kd);
}

// Parent block of one box: the children's E blocks where both points come
// from one child, generated kernel entries where they come from different
// children.
template <typename TS, typename TD, bool CPLX>
__device__ inline void assemble_box(TD* __restrict__ F, const TS* __restrict__ Fc,
                                    const BoxDev* __restrict__ boxes, int box,
                                    const LayoutDev* __restrict__ layouts, const int* __restrict__ lu,
                                    const int* __restrict__ lv, const int* __restrict__ src_c,
                                    const int* __restrict__ src_i, const KernelDesc& kd) {
    const BoxDev b = boxes[box];
    const LayoutDev L = layouts[b.layout];
    const int m = L.k + L.r;
    const BoxDev c0 = boxes[b.child0], c1 = boxes[b.child1];
    const int m0 = c0.k + c0.r, m1 = c1.k + c1.r;
    TD* Fb = F + b.offF;
    const int* U = lu + L.off_uv;
    const int* V = lv + L.off_uv;
    const int* SC = src_c + L.off_uv;
    const int* SI = src_i + L.off_uv;
    const int64_t stride_ = (int64_t)gridDim.x * 256;
    if ((int64_t)m * m > 0)
    for (ColWalk w(blockIdx.x * 256 + threadIdx.x, stride_, m); w.e < (int64_t)m * m; w.next(stride_)) {
        const int64_t e = w.e;
        const int i = w.i, j = w.j;
        const int ci = SC[i], cj = SC[j];
        TD val;
        if (ci == cj) {
            const BoxDev& c = ci ? c1 : c0;
            const int mc = ci ? m1 : m0;
            val = (TD)Fc[c.offF + SI[i] + (int64_t)SI[j] * mc];
        } else if constexpr (CPLX) {
            val = TD(cplx_entry(kd, U[i] - U[j], V[i] - V[j], 0, dof_plane(i, L.k, L.r),
                                dof_plane(j, L.k, L.r), kd.h * kd.h));
        } else {
            val = KV<TD>::off(kd, U[i] - U[j], V[i] - V[j]);
            if (kd.has_b) {
                const int64_t gi = (int64_t)(b.x0 + U[i]) * kd.ny + (b.y0 + V[i]);
                const int64_t gj = (int64_t)(b.x0 + U[j]) * kd.ny + (b.y0 + V[j]);
                val = val * TD(kd.sb[gi] * kd.sb[gj]);
            }
        }
        Fb[e] = val;
    }
}

template <typename TS, typename TD, bool CPLX>
__global__ void __launch_bounds__(256) assemble_kernel(
    TD* __restrict__ F, const TS* __restrict__ Fc, const BoxDev* __restrict__ boxes,
    const int* __restrict__ box_ids, const LayoutDev* __restrict__ layouts,
    const int* __restrict__ lu, const int* __restrict__ lv, const int* __restrict__ src_c,
    const int* __restrict__ src_i, KernelDesc kd) {
    assemble_box<TS, TD, CPLX>(F, Fc, boxes, box_ids[blockIdx.y], layouts, lu, lv, src_c, src_i, kd);
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256) assemble_group_kernel(const AsmInst* __restrict__ insts,
                                                              const GroupItem* __restrict__ items) {
    const GroupItem it = items[blockIdx.y];
    const AsmInst& I = insts[it.inst];
    assemble_box<TS, TD, false>(static_cast<TD*>(I.F), static_cast<const TS*>(I.Fc), I.boxes, it.box, I.layouts,
                         I.lu, I.lv, I.src_c, I.src_i, I.kd);
}

// Proxy matrix [K(Z, X^sk) | K(Z, X^rs)] of every interpolation problem
// (p x (k + r), ld p).  geo per problem: ax, ay, sector ab, group.  For a
// symmetry sector ab (>= 0) rows and columns are orbit representatives and
// an entry is the sector's block of the kernel in the symmetry-adapted
// basis: sum over the reflections g of the group (bit 0: u, bit 1: v) of
// (-1)^(a gx + b gy) K(z - g x), evaluated in float64.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) proxy_kernel(
    T* __restrict__ A, const int64_t* __restrict__ offA, const int* __restrict__ p_of,
    const int* __restrict__ k_of, const int* __restrict__ r_of, const int* __restrict__ zoff,
    const int* __restrict__ zu, const int* __restrict__ zv, const int* __restrict__ xoff,
    const int* __restrict__ xu, const int* __restrict__ xv, const int* __restrict__ geo,
    const double* __restrict__ logh_of, KernelDesc kdc) {
    const int pb = blockIdx.y;
    KernelDesc kd = kdc;
    if (logh_of) kd.logh = logh_of[pb];   // problems of grids with different spacings
    const int p = p_of[pb], n = k_of[pb] + r_of[pb];
    const int ax = geo[5 * pb], ay = geo[5 * pb + 1], sec = geo[5 * pb + 2], grp = geo[5 * pb + 3];
    const int prow = geo[5 * pb + 4];   // kernel rows; the rows below them (damping) start at zero
    T* Ab = A + offA[pb];
    const int* ZU = zu + zoff[pb];
    const int* ZV = zv + zoff[pb];
    const int* XU = xu + xoff[pb];
    const int* XV = xv + xoff[pb];
    const int pz = CPLX ? prow / 2 : prow;    // proxy points (rows: plane 0 then plane 1)
    const int64_t stride_ = (int64_t)gridDim.x * 256;
    if ((int64_t)p * n > 0)
    for (ColWalk w(blockIdx.x * 256 + threadIdx.x, stride_, p); w.e < (int64_t)p * n; w.next(stride_)) {
        const int64_t e = w.e;
        const int i = w.i, j = w.j;
        if (i >= prow) {
            Ab[e] = T(0);
            continue;
        }
        if constexpr (CPLX) {
            const int zi = i % pz;
            Ab[e] = T(cplx_entry(kd, ZU[zi] - XU[j], ZV[zi] - XV[j], 0, i / pz,
                                 dof_plane(j, k_of[pb], r_of[pb]), 1.0));
            continue;
        }
        if (sec < 0) {
            Ab[e] = KV<T>::proxy(kd, ZU[i] - XU[j], ZV[i] - XV[j]);
        } else {
            const int u = XU[j], v = XV[j], um = ax - 1 - u, vm = ay - 1 - v;
            const double sa = (sec & 1) ? -1.0 : 1.0, sb = (sec & 2) ? -1.0 : 1.0;
            double val = KV<double>::proxy(kd, ZU[i] - u, ZV[i] - v);
            if (grp & 1) val += sa * KV<double>::proxy(kd, ZU[i] - um, ZV[i] - v);
            if (grp & 2) val += sb * KV<double>::proxy(kd, ZU[i] - u, ZV[i] - vm);
            if (grp == 3) val += sa * sb * KV<double>::proxy(kd, ZU[i] - um, ZV[i] - vm);
            Ab[e] = T(val);
        }
    }
}

// T of a box type from float64 solutions in the sector arena, converted to
// the level's precision.  Symmetric type (d.sym) with a reflection group of
// order ns (2 or 4): from its sector solutions T^ab (orbit indices), T[i, j]
// = 1/ns sum_ab chi_ab(g_i) chi_ab(h_j) T^ab[orb_i, orb_j] over the group's
// characters ab, chi_ab(g) = (-1)^popcount(ab & g) (the symmetry-adapted
// basis is orthonormal); otherwise a plain copy.
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) sym_combine_kernel(TD* __restrict__ Ta, const TS* __restrict__ Ts,
                                                          const SymCombineDesc* __restrict__ descs,
                                                          const int* __restrict__ orb,
                                                          const int* __restrict__ refl) {
    const SymCombineDesc d = descs[blockIdx.y];
    TD* __restrict__ Tb = d.dst ? static_cast<TD*>(d.dst) : Ta + d.offT;
    const int ns = d.grp == 3 ? 4 : 2;
    const int kq = d.k / ns, rq = d.r / ns;
    const int64_t blk = (int64_t)kq * rq;
    const TS scale = TS(1) / TS(ns);
    const int64_t stride_ = (int64_t)gridDim.x * 256;
    if ((int64_t)d.k * d.r > 0)
    for (ColWalk w(blockIdx.x * 256 + threadIdx.x, stride_, d.k); w.e < (int64_t)d.k * d.r; w.next(stride_)) {
        const int64_t e = w.e;
        const int i = w.i, j = w.j;
        if (!d.sym) {
            Tb[e] = TD(Ts[d.offS + e]);
            continue;
        }
        const int oi = orb[d.off_sk + i], gi = refl[d.off_sk + i];
        const int oj = orb[d.off_rs + j], gj = refl[d.off_rs + j];
        const int64_t at = oi + (int64_t)oj * kq;
        TS acc = TS(0);
        for (int sc = 0; sc < ns; ++sc) {
            const int ab = d.grp == 2 ? 2 * sc : sc;   // sector sc's character
            const TS v = Ts[d.offS + sc * blk + at];
            acc += (__popc(ab & (gi ^ gj)) & 1) ? -v : v;
        }
        Tb[i + (int64_t)j * d.k] = TD(scale * acc);
    }
}

// F'_rs = (F'_sr)^T for one box (32 x 32 tiles through LDS)
template <typename T>
__device__ inline void transpose_box(T* __restrict__ F, const BoxDev* __restrict__ boxes, int box) {
    const BoxDev b = boxes[box];
    const int k = b.k, r = b.r, m = k + r;
    __shared__ T tile[32][33];
    const int tiles_k = (k + 31) / 32, tiles_r = (r + 31) / 32;
    T* Fb = F + b.offF;
    for (int tt = blockIdx.x; tt < tiles_k * tiles_r; tt += gridDim.x) {
        const int tk = tt % tiles_k, tr = tt / tiles_k;
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int i = e % 32, j = e / 32;
            const int gi = tk * 32 + i, gj = tr * 32 + j;
            tile[j][i] = (gi < k && gj < r) ? Fb[gi + (int64_t)(k + gj) * m] : T(0);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int j = e % 32, i = e / 32;
            const int gi = tk * 32 + i, gj = tr * 32 + j;
            if (gi < k && gj < r) Fb[(k + gj) + (int64_t)gi * m] = tile[j][i];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) transpose_kernel(T* __restrict__ F, const BoxDev* __restrict__ boxes,
                                                         const int* __restrict__ ids) {
    transpose_box<T>(F, boxes, ids[blockIdx.y]);
}

template <typename T>
__global__ void __launch_bounds__(256) transpose_group_kernel(const AsmInst* __restrict__ insts,
                                                               const GroupItem* __restrict__ items) {
    const GroupItem it = items[blockIdx.y];
    transpose_box<T>(static_cast<T*>(insts[it.inst].F), insts[it.inst].boxes, it.box);
}

inline int chunks_for(int64_t elems) {
    int64_t c = (elems + 256 * 8 - 1) / (256 * 8);
    if (c < 1) c = 1;
    if (c > 4096) c = 4096;
    return (int)c;
}

}  // namespace

template <typename T>
void launch_leaf_F(T* F, const BoxDev* boxes, const int* box_ids, int n_boxes,
                   const LayoutDev* layouts, const int* lu, const int* lv, KernelDesc kd,
                   int max_m, hipStream_t s) {
    if (n_boxes <= 0) return;
    dim3 grid(chunks_for((int64_t)max_m * max_m), n_boxes);
    if (kd.cplx)
        hipLaunchKernelGGL((leaf_F_kernel<T, true>), grid, dim3(256), 0, s, F, boxes, box_ids, layouts, lu, lv, kd);
    else
        hipLaunchKernelGGL((leaf_F_kernel<T, false>), grid, dim3(256), 0, s, F, boxes, box_ids, layouts, lu, lv, kd);
}

template <typename TS, typename TD>
void launch_assemble_F(TD* F, const TS* Fchild, const BoxDev* boxes, const int* box_ids,
                       int n_boxes, const LayoutDev* layouts, const int* lu, const int* lv,
                       const int* src_c, const int* src_i, KernelDesc kd, int max_m,
                       hipStream_t s) {
    if (n_boxes <= 0) return;
    dim3 grid(chunks_for((int64_t)max_m * max_m), n_boxes);
    if (kd.cplx)
        hipLaunchKernelGGL((assemble_kernel<TS, TD, true>), grid, dim3(256), 0, s, F, Fchild, boxes, box_ids,
                           layouts, lu, lv, src_c, src_i, kd);
    else
        hipLaunchKernelGGL((assemble_kernel<TS, TD, false>), grid, dim3(256), 0, s, F, Fchild, boxes, box_ids,
                           layouts, lu, lv, src_c, src_i, kd);
}

template <typename T>
void launch_proxy_matrix(T* A, const int64_t* offA, const int* p_of, const int* k_of,
                         const int* r_of, const int* zoff, const int* zu, const int* zv,
                         const int* xoff, const int* xu, const int* xv, const int* geo,
                         const double* logh_of, int n_problems, int max_pn, KernelDesc kd,
                         hipStream_t s) {
    if (n_problems <= 0) return;
    dim3 grid(chunks_for(max_pn), n_problems);
    if (kd.cplx)
        hipLaunchKernelGGL((proxy_kernel<T, true>), grid, dim3(256), 0, s, A, offA, p_of, k_of, r_of, zoff, zu,
                           zv, xoff, xu, xv, geo, logh_of, kd);
    else
        hipLaunchKernelGGL((proxy_kernel<T, false>), grid, dim3(256), 0, s, A, offA, p_of, k_of, r_of, zoff, zu,
                           zv, xoff, xu, xv, geo, logh_of, kd);
}

template <typename TS, typename TD>
void launch_sym_combine(TD* Tarena, const TS* Tsec, const SymCombineDesc* d, int n_desc,
                        const int* orb, const int* refl, int max_kr, hipStream_t s) {
    if (n_desc <= 0) return;
    dim3 grid(chunks_for(max_kr), n_desc);
    hipLaunchKernelGGL((sym_combine_kernel<TS, TD>), grid, dim3(256), 0, s, Tarena, Tsec, d, orb, refl);
}
template void launch_sym_combine<double, double>(double*, const double*, const SymCombineDesc*, int,
                                                 const int*, const int*, int, hipStream_t);
template void launch_sym_combine<double, float>(float*, const double*, const SymCombineDesc*, int,
                                                const int*, const int*, int, hipStream_t);
template void launch_sym_combine<float, float>(float*, const float*, const SymCombineDesc*, int,
                                               const int*, const int*, int, hipStream_t);
template void launch_sym_combine<float, double>(double*, const float*, const SymCombineDesc*, int,
                                                const int*, const int*, int, hipStream_t);

template <typename T>
void launch_transpose_sr(T* F, const BoxDev* boxes, const int* ids, int n_boxes, int max_k,
                         int max_r, hipStream_t s) {
    if (n_boxes <= 0 || max_k <= 0 || max_r <= 0) return;
    int chunks = ((max_k + 31) / 32) * ((max_r + 31) / 32);
    if (chunks > 1024) chunks = 1024;
    hipLaunchKernelGGL(transpose_kernel<T>, dim3(chunks, n_boxes), dim3(256), 0, s, F, boxes, ids);
}
// grid y is limited to 65535: longer item lists go to further launches
constexpr int GROUP_MAX_Y = 65535;

template <typename T>
void launch_leaf_F_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_m, hipStream_t s) {
    for (int o = 0; o < n_items; o += GROUP_MAX_Y) {
        dim3 grid(chunks_for((int64_t)max_m * max_m), std::min(GROUP_MAX_Y, n_items - o));
        hipLaunchKernelGGL(leaf_F_group_kernel<T>, grid, dim3(256), 0, s, insts, items + o);
    }
}

template <typename TS, typename TD>
void launch_assemble_F_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_m,
                             hipStream_t s) {
    for (int o = 0; o < n_items; o += GROUP_MAX_Y) {
        dim3 grid(chunks_for((int64_t)max_m * max_m), std::min(GROUP_MAX_Y, n_items - o));
        hipLaunchKernelGGL((assemble_group_kernel<TS, TD>), grid, dim3(256), 0, s, insts, items + o);
    }
}

template <typename T>
void launch_transpose_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_k, int max_r,
                            hipStream_t s) {
    if (max_k <= 0 || max_r <= 0) return;
    const int chunks = std::min(((max_k + 31) / 32) * ((max_r + 31) / 32), 1024);
    for (int o = 0; o < n_items; o += GROUP_MAX_Y)
        hipLaunchKernelGGL(transpose_group_kernel<T>, dim3(chunks, std::min(GROUP_MAX_Y, n_items - o)), dim3(256),
                           0, s, insts, items + o);
}

template void launch_leaf_F_group<double>(const AsmInst*, const GroupItem*, int, int, hipStream_t);
template void launch_leaf_F_group<float>(const AsmInst*, const GroupItem*, int, int, hipStream_t);
template void launch_assemble_F_group<double, double>(const AsmInst*, const GroupItem*, int, int, hipStream_t);
template void launch_assemble_F_group<float, float>(const AsmInst*, const GroupItem*, int, int, hipStream_t);
template void launch_assemble_F_group<float, double>(const AsmInst*, const GroupItem*, int, int, hipStream_t);
template void launch_transpose_group<double>(const AsmInst*, const GroupItem*, int, int, int, hipStream_t);
template void launch_transpose_group<float>(const AsmInst*, const GroupItem*, int, int, int, hipStream_t);

template void launch_transpose_sr<double>(double*, const BoxDev*, const int*, int, int, int, hipStream_t);
template void launch_transpose_sr<float>(float*, const BoxDev*, const int*, int, int, int, hipStream_t);

template void launch_leaf_F<double>(double*, const BoxDev*, const int*, int, const LayoutDev*,
                                    const int*, const int*, KernelDesc, int, hipStream_t);
template void launch_leaf_F<float>(float*, const BoxDev*, const int*, int, const LayoutDev*,
                                   const int*, const int*, KernelDesc, int, hipStream_t);
template void launch_assemble_F<double, double>(double*, const double*, const BoxDev*, const int*,
                                                int, const LayoutDev*, const int*, const int*,
                                                const int*, const int*, KernelDesc, int, hipStream_t);
template void launch_assemble_F<float, float>(float*, const float*, const BoxDev*, const int*, int,
                                              const LayoutDev*, const int*, const int*, const int*,
                                              const int*, KernelDesc, int, hipStream_t);
template void launch_assemble_F<float, double>(double*, const float*, const BoxDev*, const int*, int,
                                               const LayoutDev*, const int*, const int*, const int*,
                                               const int*, KernelDesc, int, hipStream_t);
template void launch_proxy_matrix<double>(double*, const int64_t*, const int*, const int*,
                                          const int*, const int*, const int*, const int*,
                                          const int*, const int*, const int*, const int*,
                                          const double*, int, int, KernelDesc, hipStream_t);
template void launch_proxy_matrix<float>(float*, const int64_t*, const int*, const int*,
                                         const int*, const int*, const int*, const int*,
                                         const int*, const int*, const int*, const int*,
                                         const double*, int, int, KernelDesc, hipStream_t);

}  // namespace rsd
