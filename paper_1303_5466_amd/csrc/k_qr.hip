// Interpolation matrices T by column-pivoted Householder QR least squares.
//
// For each box type, T solves  K(Z, X^sk) T = K(Z, X^rs)  with Z the proxy
// ring of Sec. 3.1 (rectangular case: least squares, remark after
// Algorithm 3).  The interpolative decomposition of Sec. 2.1 is a
// column-pivoted QR truncated where |R_jj| <= tol |R_11|; the solution is
// T = Pi [R11^{-1} Q1^T K(Z, X^rs); 0].
//
// GPU formulation (all interpolation problems of all levels advance
// together, one launch per panel step):
//   qr_init    column norms of K(Z, X^sk), identity permutation;
//   qr_panel   one 1024-thread workgroup per problem: picks the QR_NB
//              columns of largest remaining norm (wavefront argmax, lowest
//              index on ties), factors that panel in registers with
//              Businger-Golub pivoting inside the panel, checks the
//              truncation rule, and forms the compact-WY factor;
//   qr_update  applies the panel's reflectors to every trailing column
//              (candidates and right-hand sides) and recomputes the exact
//              trailing norms used by the next panel's selection;
//   qr_solve   back substitution with R11 and the scatter through Pi.
// Pivoting is therefore exact within a panel and by block (largest norms
// first) across panels; see the design notes for why this replaces strict
// column-by-column pivoting.
#include "common.hpp"

namespace rsd {

namespace {

constexpr int NB = QR_NB;
constexpr int PT = 512;    // panel workgroup size

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// aux layout per problem
template <typename T> struct Aux {
    T* norms; T* tau; T* Tf; T* r11;
    int* perm; int* state;   // state: rank, nref, j0, nbe
    __device__ Aux(T* aux, int* iaux, const QRProblemDev& q) {
        norms = aux + q.offAux;
        tau = norms + q.k;
        Tf = tau + q.k;
        r11 = Tf + NB * NB;
        perm = iaux + q.offIaux;
        state = perm + q.k;
    }
};

template <typename T>
__global__ void __launch_bounds__(256) qr_init_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                       int* __restrict__ iaux,
                                                       const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, q);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + wave;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        X.state[0] = -1; X.state[1] = 0; X.state[2] = 0; X.state[3] = 0;
        X.r11[0] = T(0);
    }
    if (c >= q.k) return;
    const T* col = A + q.offA + (int64_t)c * q.p;
    T s = T(0);
    for (int i = lane; i < q.p; i += 64) s += col[i] * col[i];
    s = wave_sum(s);
    if (lane == 0) { X.norms[c] = s; X.perm[c] = c; }
}

// block-wide reduction of NV values (each thread supplies v[0..NV)), result
// broadcast to every thread in a fixed order (identical in every thread)
template <typename T, int NV>
__device__ inline void block_sum(T (&v)[NV], T* red /* [PT/64][NV] */) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) red[wave * NV + j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        T s = T(0);
        for (int w = 0; w < PT / 64; ++w) s += red[w * NV + j];
        v[j] = s;
    }
}

template <typename T, int W, int MAXR>
__global__ void __launch_bounds__(PT) qr_panel_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                       int* __restrict__ iaux,
                                                       const QRProblemDev* __restrict__ probs,
                                                       const int* __restrict__ plist, int step,
                                                       double tol) {
    const QRProblemDev q = probs[plist[blockIdx.x]];
    Aux<T> X(aux, iaux, q);
    const int t = threadIdx.x;
    __shared__ T red[(PT / 64) * W];
    __shared__ T Tfs[W][W];
    __shared__ T bx0;
    __shared__ int bidx[PT / 64];
    __shared__ T bnorm[PT / 64];
    __shared__ int lperm[W];
    __shared__ int gperm_old[W];
    const int j0 = step * W;
    if (X.state[0] >= 0 || j0 >= q.k) {
        __syncthreads();
        if (t == 0) {
            if (X.state[0] < 0) X.state[0] = q.k;
            X.state[1] = 0;
        }
        return;
    }
    const int nbe = min(W, q.k - j0);
    const int pr = q.p - j0;
    T* Ab = A + q.offA;
    // ---- (1) block selection: the nbe largest remaining column norms -----
    for (int c = 0; c < nbe; ++c) {
        T best = T(-1);
        int bi = 0x7fffffff;
        for (int j = j0 + c + t; j < q.k; j += PT) {
            const T v = X.norms[j];
            if (v > best) { best = v; bi = j; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const T ov = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if ((t & 63) == 0) { bnorm[t >> 6] = best; bidx[t >> 6] = bi; }
        __syncthreads();
        if (t == 0) {
            T b = bnorm[0];
            int i = bidx[0];
            for (int w = 1; w < PT / 64; ++w)
                if (bnorm[w] > b || (bnorm[w] == b && bidx[w] < i)) { b = bnorm[w]; i = bidx[w]; }
            bidx[0] = i;
        }
        __syncthreads();
        const int jm = bidx[0];
        const int jc = j0 + c;
        if (jm != jc) {
            T* ca = Ab + (int64_t)jc * q.p;
            T* cb = Ab + (int64_t)jm * q.p;
            for (int i = t; i < q.p; i += PT) { const T x = ca[i]; ca[i] = cb[i]; cb[i] = x; }
            if (t == 0) {
                const T x = X.norms[jc]; X.norms[jc] = X.norms[jm]; X.norms[jm] = x;
                const int y = X.perm[jc]; X.perm[jc] = X.perm[jm]; X.perm[jm] = y;
            }
        }
        __syncthreads();
    }
    // ---- (2) panel into registers: thread t holds panel rows t + s*PT ----
    T a[MAXR][W];
#pragma unroll
    for (int s = 0; s < MAXR; ++s) {
        const int i = t + s * PT;
#pragma unroll
        for (int j = 0; j < W; ++j)
            a[s][j] = (i < pr && j < nbe) ? Ab[(j0 + i) + (int64_t)(j0 + j) * q.p] : T(0);
    }
    int perm_loc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) perm_loc[j] = j;
    T taus[W];
#pragma unroll
    for (int j = 0; j < W; ++j) taus[j] = T(0);
    for (int e = t; e < W * W; e += PT) Tfs[e % W][e / W] = T(0);
    int nref = nbe;
    T r11 = step == 0 ? T(0) : X.r11[0];
    bool stop = false;
    // ---- (3) Householder QR of the panel, pivoting inside the panel ------
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (c < nbe && !stop) {
            T nrm[W];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                T s2 = T(0);
                if (j >= c) {
#pragma unroll
                    for (int s = 0; s < MAXR; ++s) {
                        const int i = t + s * PT;
                        if (i >= c && i < pr) s2 += a[s][j] * a[s][j];
                    }
                }
                nrm[j] = s2;
            }
            block_sum<T, W>(nrm, red);
            int pv = c;
            T pn = nrm[c];
#pragma unroll
            for (int j = c + 1; j < W; ++j)
                if (j < nbe && nrm[j] > pn) { pn = nrm[j]; pv = j; }
            if (pv != c) {
#pragma unroll
                for (int j = c + 1; j < W; ++j) {
                    if (j == pv) {
#pragma unroll
                        for (int s = 0; s < MAXR; ++s) { const T x = a[s][c]; a[s][c] = a[s][j]; a[s][j] = x; }
                        const int x = perm_loc[c]; perm_loc[c] = perm_loc[j]; perm_loc[j] = x;
                    }
                }
            }
            const T normx = sqrt(pn);
            if (step == 0 && c == 0) r11 = normx;
            if (!(normx > T(tol) * r11)) {
                stop = true;
                nref = c;
            } else {
                // x0 = panel row c, held by thread c (slot 0)
                if (t == c) bx0 = a[0][c];
                __syncthreads();
                const T x0 = bx0;
                const T beta = x0 >= T(0) ? -normx : normx;
                const T tau = (beta - x0) / beta;
                const T scl = T(1) / (x0 - beta);
#pragma unroll
                for (int s = 0; s < MAXR; ++s) {
                    const int i = t + s * PT;
                    if (i == c) a[s][c] = beta;
                    else if (i > c && i < pr) a[s][c] *= scl;
                }
                taus[c] = tau;
                // d[j] = v_c^T a_j (j > c); d[i] = v_i^T v_c (i < c, for the WY factor)
                T d[W];
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    T s2 = T(0);
                    if (j != c) {
#pragma unroll
                        for (int s = 0; s < MAXR; ++s) {
                            const int i = t + s * PT;
                            const T vc = (i == c) ? T(1) : ((i > c && i < pr) ? a[s][c] : T(0));
                            T other;
                            if (j > c) other = a[s][j];
                            else other = (i == j) ? T(1) : ((i > j && i < pr) ? a[s][j] : T(0));
                            s2 += vc * other;
                        }
                    }
                    d[j] = s2;
                }
                block_sum<T, W>(d, red);
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    if (j > c && j < nbe) {
                        const T f = tau * d[j];
#pragma unroll
                        for (int s = 0; s < MAXR; ++s) {
                            const int i = t + s * PT;
                            const T vc = (i == c) ? T(1) : ((i > c && i < pr) ? a[s][c] : T(0));
                            a[s][j] -= f * vc;
                        }
                    }
                }
                // compact-WY column c: Tf[0:c, c] = -tau Tf[0:c, 0:c] d[0:c]
                if (t < c) {
                    T s2 = T(0);
#pragma unroll
                    for (int l = 0; l < W; ++l)
                        if (l >= t && l < c) s2 += Tfs[t][l] * d[l];
                    Tfs[t][c] = -tau * s2;
                }
                if (t == c) Tfs[c][c] = tau;
                __syncthreads();
            }
        }
    }
    // ---- (4) write back panel, tau, permutation ---------------------------
#pragma unroll
    for (int s = 0; s < MAXR; ++s) {
        const int i = t + s * PT;
        if (i < pr)
#pragma unroll
            for (int j = 0; j < W; ++j)
                if (j < nbe) Ab[(j0 + i) + (int64_t)(j0 + j) * q.p] = a[s][j];
    }
    if (t < W) {
        lperm[t] = perm_loc[t];
        if (t < nbe) gperm_old[t] = X.perm[j0 + t];
    }
    __syncthreads();
    // rows above the panel hold earlier R entries of these columns
    for (int i = t; i < j0; i += PT) {
        T tmp[W];
#pragma unroll
        for (int j = 0; j < W; ++j) tmp[j] = j < nbe ? Ab[i + (int64_t)(j0 + j) * q.p] : T(0);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if (j < nbe) {
                T v = T(0);
#pragma unroll
                for (int jj = 0; jj < W; ++jj)
                    if (jj == lperm[j]) v = tmp[jj];
                Ab[i + (int64_t)(j0 + j) * q.p] = v;
            }
        }
    }
    if (t < nbe) {
        X.perm[j0 + t] = gperm_old[lperm[t]];
        X.tau[j0 + t] = taus[t];
    }
    for (int e = t; e < NB * NB; e += PT) {
        const int i = e % NB, j = e / NB;
        X.Tf[e] = (i < W && j < W && i < nref && j < nref) ? Tfs[i][j] : T(0);
    }
    if (t == 0) {
        if (step == 0) X.r11[0] = r11;
        X.state[1] = nref;
        X.state[2] = j0;
        X.state[3] = nbe;
        if (nref < nbe) X.state[0] = j0 + nref;
        else if (j0 + nbe >= q.k) X.state[0] = q.k;
    }
}

// Apply the panel reflectors to the trailing columns [j0 + nbe, k + r) and
// recompute trailing norms (rows >= j0 + nref) of candidate columns.
template <typename T>
__global__ void __launch_bounds__(256) qr_update_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                         int* __restrict__ iaux,
                                                         const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, q);
    const int nref = X.state[1];
    if (nref == 0) return;
    const int j0 = X.state[2], nbe = X.state[3];
    const int n = q.k + q.r;
    const int cstart = j0 + nbe + blockIdx.x * 16;
    if (cstart >= n) return;
    const int pr = q.p - j0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* Ab = A + q.offA;
    __shared__ T Vs[64][NB + 1];
    __shared__ T Tf[NB][NB];
    for (int e = threadIdx.x; e < NB * NB; e += 256) Tf[e % NB][e / NB] = X.Tf[e];
    T acc[4][NB];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[cc][j] = T(0);
    // pass 1: W = V^T A_slab
    for (int r0 = 0; r0 < pr; r0 += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * NB; e += 256) {
            const int i = e & 63, j = e >> 6;
            const int r = r0 + i;
            T v = T(0);
            if (j < nref && r < pr) v = (r == j) ? T(1) : (r > j ? Ab[(j0 + r) + (int64_t)(j0 + j) * q.p] : T(0));
            Vs[i][j] = v;
        }
        __syncthreads();
        const int r = r0 + lane;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int col = cstart + wave + 4 * cc;
            if (col < n && r < pr) {
                const T x = Ab[(j0 + r) + (int64_t)col * q.p];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[cc][j] += Vs[lane][j] * x;
            }
        }
    }
    // reduce over lanes, then W' = Tf^T W
    T wv[4][NB];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[cc][j] = wave_sum(acc[cc][j]);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            T s2 = T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i <= j) s2 += Tf[i][j] * acc[cc][i];
            wv[cc][j] = j < nref ? s2 : T(0);
        }
    }
    // pass 2: A_slab -= V W', trailing norms
    T nr[4] = {T(0), T(0), T(0), T(0)};
    for (int r0 = 0; r0 < pr; r0 += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * NB; e += 256) {
            const int i = e & 63, j = e >> 6;
            const int r = r0 + i;
            T v = T(0);
            if (j < nref && r < pr) v = (r == j) ? T(1) : (r > j ? Ab[(j0 + r) + (int64_t)(j0 + j) * q.p] : T(0));
            Vs[i][j] = v;
        }
        __syncthreads();
        const int r = r0 + lane;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int col = cstart + wave + 4 * cc;
            if (col < n && r < pr) {
                T* px = Ab + (j0 + r) + (int64_t)col * q.p;
                T x = *px;
#pragma unroll
                for (int j = 0; j < NB; ++j) x -= Vs[lane][j] * wv[cc][j];
                *px = x;
                if (r >= nref) nr[cc] += x * x;
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        const T s2 = wave_sum(nr[cc]);
        const int col = cstart + wave + 4 * cc;
        if (lane == 0 && col < q.k) X.norms[col] = s2;
    }
}

// R11 X = (Q^T K(Z, X^rs))[0:rank, :], then T[perm[i], :] = X[i, :].
template <typename T>
__global__ void __launch_bounds__(256) qr_solve_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                        int* __restrict__ iaux, T* __restrict__ Tout,
                                                        const QRProblemDev* __restrict__ probs,
                                                        int cols_per_wg) {
    extern __shared__ unsigned char smem_raw[];
    T* xs = reinterpret_cast<T*>(smem_raw);
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, q);
    const int rank = X.state[0] < 0 ? q.k : X.state[0];
    const int c0 = blockIdx.x * cols_per_wg;
    if (c0 >= q.r) return;
    const int nc = min(cols_per_wg, q.r - c0);
    const T* Ab = A + q.offA;
    for (int e = threadIdx.x; e < rank * nc; e += 256) {
        const int i = e % rank, c = e / rank;
        xs[i + c * rank] = Ab[i + (int64_t)(q.k + c0 + c) * q.p];
    }
    __syncthreads();
    for (int i = rank - 1; i >= 0; --i) {
        const T* Ri = Ab + (int64_t)i * q.p;     // column i of R
        const T rii = Ri[i];
        for (int c = 0; c < nc; ++c) {
            const T xi = xs[i + c * rank] / rii;
            for (int l = threadIdx.x; l < i; l += 256) xs[l + c * rank] -= xi * Ri[l];
        }
        __syncthreads();
        if (threadIdx.x < nc) xs[i + threadIdx.x * rank] = xs[i + threadIdx.x * rank] / rii;
        __syncthreads();
    }
    T* To = Tout + q.offT;
    for (int e = threadIdx.x; e < q.k * nc; e += 256) {
        const int i = e % q.k, c = e / q.k;
        const T v = i < rank ? xs[i + c * rank] : T(0);
        To[X.perm[i] + (int64_t)(c0 + c) * q.k] = v;
    }
}

}  // namespace

template <typename T>
void launch_qr_init(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int max_k,
                    hipStream_t s) {
    if (n_probs <= 0) return;
    hipLaunchKernelGGL(qr_init_kernel<T>, dim3((max_k + 3) / 4, n_probs), dim3(256), 0, s, A, aux,
                       iaux, probs);
}

int qr_panel_width(int p) {
    if (p <= 2 * PT * 2) return 16;      // MAXR 4
    if (p <= 8 * PT) return 8;           // MAXR 8
    if (p <= 16 * PT) return 4;          // MAXR 16
    return 0;
}

template <typename T>
void launch_qr_panel(T* A, T* aux, int* iaux, const QRProblemDev* probs, const int* plist,
                     int n_list, int nb_class, int step, double tol, hipStream_t s) {
    if (n_list <= 0) return;
    if (nb_class == 16)
        hipLaunchKernelGGL((qr_panel_kernel<T, 16, 4>), dim3(n_list), dim3(PT), 0, s, A, aux, iaux, probs, plist, step, tol);
    else if (nb_class == 8)
        hipLaunchKernelGGL((qr_panel_kernel<T, 8, 8>), dim3(n_list), dim3(PT), 0, s, A, aux, iaux, probs, plist, step, tol);
    else if (nb_class == 4)
        hipLaunchKernelGGL((qr_panel_kernel<T, 4, 16>), dim3(n_list), dim3(PT), 0, s, A, aux, iaux, probs, plist, step, tol);
    else
        throw HipError("interpolation problem too large for the panel kernel");
}

template <typename T>
void launch_qr_update(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int step,
                      int max_n, hipStream_t s) {
    if (n_probs <= 0) return;
    (void)step;
    hipLaunchKernelGGL(qr_update_kernel<T>, dim3((max_n + 15) / 16, n_probs), dim3(256), 0, s, A,
                       aux, iaux, probs);
}

template <typename T>
void launch_qr_solve(T* A, T* aux, int* iaux, T* Tout, const QRProblemDev* probs, int n_probs,
                     int max_r, int max_k, hipStream_t s) {
    if (n_probs <= 0 || max_r <= 0) return;
    const int budget = 60 * 1024;
    int cols = budget / (int)(sizeof(T) * (max_k > 0 ? max_k : 1));
    if (cols > 8) cols = 8;
    if (cols < 1) throw HipError("interpolation problem too large for the solve kernel");
    const size_t shm = sizeof(T) * (size_t)max_k * cols;
    hipLaunchKernelGGL(qr_solve_kernel<T>, dim3((max_r + cols - 1) / cols, n_probs), dim3(256), shm,
                       s, A, aux, iaux, Tout, probs, cols);
}

#define INST(T)                                                                                   \
    template void launch_qr_init<T>(T*, T*, int*, const QRProblemDev*, int, int, hipStream_t);     \
    template void launch_qr_panel<T>(T*, T*, int*, const QRProblemDev*, const int*, int, int, int, \
                                     double, hipStream_t);                                        \
    template void launch_qr_update<T>(T*, T*, int*, const QRProblemDev*, int, int, int,            \
                                      hipStream_t);                                               \
    template void launch_qr_solve<T>(T*, T*, int*, T*, const QRProblemDev*, int, int, int,         \
                                     hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace rsd
