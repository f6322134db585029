// Interpolation matrices T by column-pivoted Householder QR least squares.
//
// For each box type, T solves  K(Z, X^sk) T = K(Z, X^rs)  with Z the proxy
// ring of Sec. 3.1 (rectangular case: least squares, remark after
// Algorithm 3).  The interpolative decomposition of Sec. 2.1 is a
// column-pivoted QR truncated where |R_jj| <= tol |R_11|; the solution is
// T = Pi [R11^{-1} Q1^T K(Z, X^rs); 0].
//
// GPU formulation: a blocked Householder QR whose pivoting is exact inside
// a window of QR_WIN columns and by block across windows.  All problems of
// all levels advance together; per window:
//   qr_select   the QR_WIN candidates of largest exact trailing norm
//               (wavefront argmax, lowest index on ties) and the column
//               moves that bring them to the window, in that order;
//   qr_move     the moves (staged through a buffer, so any permutation);
//   qr_panel    sub-panels of 16/8/4 columns factored in LDS with
//               Businger-Golub pivoting and the truncation rule
//               |R_jj| <= tol |R_11|, reflectors copied to a V workspace;
//   qr_inner    each sub-panel's reflectors applied to the rest of the window;
//   trailing    W = V^T [V | C] by split-K MFMA GEMMs, qr_wsum / qr_tbuild
//               reduce it and form the window's compact-WY factor, then
//               C -= V (Tw^T W) as two more GEMMs (the grouped GEMM kernel);
//   qr_norms    exact trailing norms for the next window.
// qr_trsm finally back-substitutes with R11, one 64-row block per call with
// the rows above updated by grouped GEMMs in between, and scatters through Pi.
#include <map>
#include <type_traits>
#include <mutex>

#include "common.hpp"

namespace rsd {

namespace {

constexpr int NB = QR_NB;
constexpr int WIN = QR_WIN;
constexpr int PT = 512;

__device__ inline float read_lane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double read_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Value of the partner lane l ^ m, with m = 1, 2, 7, 8, 16, 32 for b = 0..5:
// quad permutes, row half-mirror and row rotate-by-8 through DPP, then the
// gfx950 row-pair and half-wave swaps (each returns both halves; the lane
// keeps the other one).  All register to register.
__device__ inline int xchg_i(int x, int b) {
    const int lane = threadIdx.x & 63;
    switch (b) {
        case 0: return __builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false);   // quad_perm 1,0,3,2
        case 1: return __builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false);   // quad_perm 2,3,0,1
        case 2: return __builtin_amdgcn_update_dpp(0, x, 0x141, 0xf, 0xf, false);  // row_half_mirror
        case 3: return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false);  // row_ror:8
        case 4: {
            const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
            return (lane & 16) ? (int)r[0] : (int)r[1];
        }
        default: {
            const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
            return (lane & 32) ? (int)r[0] : (int)r[1];
        }
    }
}
__device__ inline float xchg(float v, int b) { return __int_as_float(xchg_i(__float_as_int(v), b)); }
__device__ inline double xchg(double v, int b) {
    const int lo = xchg_i(__double2loint(v), b), hi = xchg_i(__double2hiint(v), b);
    return __hiloint2double(hi, lo);
}

// Wave-wide sum by a butterfly over the six exchanges: every lane ends with
// the same (bitwise) total.
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int b = 0; b < 6; ++b) v += xchg(v, b);
    return v;
}

// Per-problem state: physical column order equals pivoted order; perm holds
// the original column index of each position.
template <typename T> struct Aux {
    T* norms; T* tau; T* Tf; T* Tw; T* r11;
    int* perm; int* state;   // state: rank, skip, J0, WO, nref, nmoves, j0, nbe
    int* moves;              // (src, dst) pairs
    T* V; T* Tmp; T* Wp; T* Ws;
    __device__ Aux(T* aux, int* iaux, T* ws, const QRProblemDev& q) {
        norms = aux + q.offAux;
        tau = norms + q.k;
        Tf = tau + q.k;
        Tw = Tf + NB * NB;
        r11 = Tw + WIN * WIN;
        perm = iaux + q.offIaux;
        state = perm + q.k;
        moves = state + 8;
        V = ws ? ws + q.offV : nullptr;
        Tmp = ws ? ws + q.offTmp : nullptr;
        Wp = ws ? ws + q.offW : nullptr;
        Ws = ws ? ws + q.offWs : nullptr;
    }
};

template <typename T>
__global__ void __launch_bounds__(256) qr_init_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                       int* __restrict__ iaux,
                                                       const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, nullptr, q);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + wave;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < 8; ++i) X.state[i] = 0;
        X.state[0] = -1;
        X.r11[0] = T(0);
    }
    if (c >= q.k) return;
    const T* col = A + q.offA + (int64_t)c * q.p;
    T s = T(0);
    for (int i = lane; i < q.p; i += 64) s += col[i] * col[i];
    s = wave_sum(s);
    if (lane == 0) { X.norms[c] = s; X.perm[c] = c; }
}

// Reference pivot of the truncation rule |R_jj| <= tol |R_11|: the largest
// column norm of the problem, or, for the sectors of a symmetric problem
// (two or four, consecutive in the list from g0), the largest over all of
// them, so that a split problem truncates against the same scale as the
// whole one.  The host checks every group against the list before launch.
template <typename T>
__global__ void __launch_bounds__(256) qr_r11_kernel(T* __restrict__ aux, int* __restrict__ iaux,
                                                      const QRProblemDev* __restrict__ probs) {
    const int pi = blockIdx.x;
    const QRProblemDev q = probs[pi];
    const int first = q.g0, count = q.gn;
    T m = T(0);
    for (int g = 0; g < count; ++g) {
        const QRProblemDev qg = probs[first + g];
        Aux<T> Y(aux, iaux, nullptr, qg);
        for (int c = threadIdx.x; c < qg.k; c += 256) m = fmax(m, Y.norms[c]);
    }
    __shared__ T red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Aux<T> X(aux, iaux, nullptr, q);
        X.r11[0] = sqrt(red[0]);
        if (q.rec) {
            q.rec[1] = (double)X.r11[0];
            q.rec[2] = (double)q.gn;
        }
    }
}

// Damped least squares: row pz + j of column j takes lambda = damp |R_11|
// (the rows were zero so far), and the column's squared norm grows by
// lambda^2.  The problem becomes min |K T - B|^2 + lambda^2 |T|^2, whose R
// has no pivot below lambda.
template <typename T>
__global__ void __launch_bounds__(256) qr_damp_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                       int* __restrict__ iaux,
                                                       const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    if (!(q.damp > 0)) return;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q.k || q.pz + j >= q.p) return;
    Aux<T> X(aux, iaux, nullptr, q);
    const T lam = T(q.damp) * X.r11[0];
    A[q.offA + (q.pz + j) + (int64_t)j * q.p] = lam;
    X.norms[j] += lam * lam;
}

// Window selection and the permutation that realises it.  The remaining
// candidates are ordered by (trailing norm descending, column ascending) with
// a bitonic sort in LDS (nsort, a power of two at least the number of
// candidates, padded with keys below every norm); the first QR_WIN entries
// are the window, in that order.  The moves are then derived by wave 0.
// K: the sort key type, T, or float where T keys would not fit the LDS (the
// largest problems; the order then follows the norms rounded to float).
template <typename T, typename K = T>
__global__ void __launch_bounds__(256) qr_select_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                         int* __restrict__ iaux, T* __restrict__ ws,
                                                         const QRProblemDev* __restrict__ probs,
                                                         int outer, int nsort) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    K* key = reinterpret_cast<K*>(smem_raw);
    int* idx = reinterpret_cast<int*>(key + nsort);
    const QRProblemDev q = probs[blockIdx.x];
    Aux<T> X(aux, iaux, ws, q);
    const int t = threadIdx.x, lane = t & 63;
    const bool w0 = t < 64;
    __shared__ int chosen[WIN];
    __shared__ int inwin[WIN];
    __shared__ int mv[4 * WIN];
    __shared__ T nv[2 * WIN];
    __shared__ int pv[2 * WIN];
    __shared__ int dlist[WIN], olist[WIN];
    const int J0 = outer * WIN;
    int skip = 0;
    if (X.state[0] >= 0) skip = 1;
    else if (J0 >= q.k) skip = 2;
    __syncthreads();
    if (t == 0) {
        if (skip == 2) X.state[0] = q.k;
        X.state[1] = skip ? 1 : 0;
        X.state[5] = 0;
    }
    if (skip) return;
    const int WO = min(WIN, q.k - J0);
    const int nrem = q.k - J0;
    for (int i = t; i < nsort; i += 256) {
        key[i] = i < nrem ? K(X.norms[J0 + i]) : K(-1);
        idx[i] = i;
    }
    if (t < WIN && J0 + t < q.k) X.tau[J0 + t] = T(0);
    if (w0) inwin[lane] = 0;
    __syncthreads();
    for (int size = 2; size <= nsort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = t; e < (nsort >> 1); e += 256) {
                const int i = 2 * stride * (e / stride) + (e % stride), j = i + stride;
                const K ki = key[i], kj = key[j];
                const int ii = idx[i], ij = idx[j];
                // does j belong before i?
                const bool jfirst = kj > ki || (kj == ki && ij < ii);
                const bool swap = ((i & size) == 0) ? jfirst : !jfirst;
                if (swap) { key[i] = kj; key[j] = ki; idx[i] = ij; idx[j] = ii; }
            }
            __syncthreads();
        }
    }
    if (t < WO) chosen[t] = idx[t];
    __syncthreads();
    // slot c <- chosen[c]; displaced window columns -> the outside chosen slots
    const int ch = (w0 && lane < WO) ? chosen[lane] : -1;
    if (w0 && lane < WO && ch < WO) inwin[ch] = 1;
    __syncthreads();
    const bool disp = w0 && lane < WO && !inwin[lane];
    const bool outc = w0 && lane < WO && ch >= WO;
    const bool mov = w0 && lane < WO && ch != lane;
    const unsigned long long bd = __ballot(disp), bo = __ballot(outc), bm = __ballot(mov);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nmove1 = __popcll(bm);
    const int i1 = __popcll(bm & below);
    if (mov) { mv[2 * i1] = J0 + ch; mv[2 * i1 + 1] = J0 + lane; }
    // pair the j-th displaced slot with the j-th outside chosen slot
    if (disp) dlist[__popcll(bd & below)] = lane;
    if (outc) olist[__popcll(bo & below)] = ch;
    __syncthreads();
    const int nd = __popcll(bd);
    if (w0 && lane < nd) { mv[2 * (nmove1 + lane)] = J0 + dlist[lane]; mv[2 * (nmove1 + lane) + 1] = J0 + olist[lane]; }
    __syncthreads();
    if (!w0) return;
    const int nm = nmove1 + nd;
    for (int m = lane; m < nm; m += 64) { nv[m] = X.norms[mv[2 * m]]; pv[m] = X.perm[mv[2 * m]]; }
    for (int m = lane; m < nm; m += 64) {   // each lane re-reads only what it staged
        X.norms[mv[2 * m + 1]] = nv[m];
        X.perm[mv[2 * m + 1]] = pv[m];
        X.moves[2 * m] = mv[2 * m];
        X.moves[2 * m + 1] = mv[2 * m + 1];
    }
    if (lane == 0) { X.state[2] = J0; X.state[3] = WO; X.state[5] = nm; }
}

// phase 0: stage the source columns of the moves; phase 1: write them to their slots
template <typename T>
__global__ void __launch_bounds__(256) qr_move_kernel(T* __restrict__ A, int* __restrict__ iaux,
                                                       T* __restrict__ ws,
                                                       const QRProblemDev* __restrict__ probs,
                                                       int phase) {
    const QRProblemDev q = probs[blockIdx.y];
    const int* state = iaux + q.offIaux + q.k;
    if (state[1]) return;
    const int m = blockIdx.x;
    if (m >= 2 * WIN) {                 // phase 0 only: clear one V column of the window
        T* v = ws + q.offV + (int64_t)(m - 2 * WIN) * q.p;
        for (int i = threadIdx.x; i < q.p; i += 256) v[i] = T(0);
        return;
    }
    if (m >= state[5]) return;
    const int* moves = state + 8;
    T* tmp = ws + q.offTmp + (int64_t)m * q.p;
    T* Ab = A + q.offA;
    if (phase == 0) {
        const T* src = Ab + (int64_t)moves[2 * m] * q.p;
        for (int i = threadIdx.x; i < q.p; i += 256) tmp[i] = src[i];
    } else {
        T* dst = Ab + (int64_t)moves[2 * m + 1] * q.p;
        for (int i = threadIdx.x; i < q.p; i += 256) dst[i] = tmp[i];
    }
}

// Block-wide sums of N values per thread (N a power of two, at most 64),
// returned in every thread in the same order.  Within a wave a butterfly
// halves the values held per lane at each exchange (lanes on the set side of
// the exchange keep the upper half), so N values cost N - 1 + 6 - log2 N
// register exchanges instead of 6 N; the four wave partials meet in LDS.
// red alternates between two halves (parity) so that one barrier per call
// suffices.
// An empty asm statement the optimiser cannot look through: it keeps a
// select between two register-array elements from being rewritten as an
// indexed load, which would move the whole array to scratch memory.
__device__ inline void opaque(double& x) { asm("" : "+v"(x)); }
__device__ inline void opaque(float& x) { asm("" : "+v"(x)); }

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int N> struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

template <typename T, int N, int RS>
__device__ inline const T* block_sum_n(T (&v)[N], T* red /* [2][RS] */, int& parity) {
    constexpr int LN = Log2<N>::v;
    static_assert((1 << LN) == N && LN <= 6 && N * (PT / 64 + 1) <= RS, "power of two up to 64");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < LN; ++s) {
        const int b = 5 - s;                    // exchange b flips lane bit b (and lower ones)
        const bool hi = (lane >> b) & 1;
        const int h = N >> (s + 1);
#pragma unroll
        for (int j = 0; j < N / 2; ++j) {
            if (j < h) {
                T lo_v = v[j], hi_v = v[j + h];
                opaque(lo_v);
                opaque(hi_v);   // keeps the selects on values, not on array slots
                const T send = hi ? lo_v : hi_v;
                const T keep = hi ? hi_v : lo_v;
                v[j] = keep + xchg(send, b);
            }
        }
    }
#pragma unroll
    for (int b = 5 - LN; b >= 0; --b) v[0] += xchg(v[0], b);
    T* r = red + parity * RS;
    if ((lane & ((64 >> LN) - 1)) == 0) r[(lane >> (6 - LN)) * (PT / 64) + wave] = v[0];
    __syncthreads();
    // thread j < N adds the wave partials of value j (fixed order, so every
    // thread gets the same bits), then every thread reads the N totals
    T* tot = r + N * (PT / 64);
    if (threadIdx.x < N) {
        T s2 = T(0);
#pragma unroll
        for (int w = 0; w < PT / 64; ++w) s2 += r[threadIdx.x * (PT / 64) + w];
        tot[threadIdx.x] = s2;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = tot[j];
    parity ^= 1;
    return r;   // the wave partials of value j at r[j * (PT / 64) + w]
}

// Sub-panel rows in LDS: row-major, W entries per row, the row stride padded
// to 4 (mod 8) dwords so that 16-byte row reads by consecutive lanes are
// free of bank conflicts; single columns (W = 1, the largest problems) are
// read one element per lane and stored unpadded.
template <typename T, int W>
constexpr int panel_stride() {
    if (W == 1) return 1;
    int s = (int)(W * sizeof(T) / 4);
    while (s % 8 != 4) ++s;
    return s * 4 / (int)sizeof(T);
}

template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct Vec16<float> { typedef float __attribute__((ext_vector_type(4))) type; };

template <typename T, int W>
__device__ inline void load_row(const T* p, T (&x)[W]) {
    constexpr int n = 16 / sizeof(T);
    if constexpr (W % n == 0) {
        typedef typename Vec16<T>::type V;
#pragma unroll
        for (int j = 0; j < W / n; ++j) {
            const V v = reinterpret_cast<const V*>(p)[j];
#pragma unroll
            for (int e = 0; e < n; ++e) x[j * n + e] = v[e];
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) x[j] = p[j];
    }
}

template <typename T, int W>
__device__ inline void store_row(T* p, const T (&x)[W]) {
    constexpr int n = 16 / sizeof(T);
    if constexpr (W % n == 0) {
        typedef typename Vec16<T>::type V;
#pragma unroll
        for (int j = 0; j < W / n; ++j) {
            V v;
#pragma unroll
            for (int e = 0; e < n; ++e) v[e] = x[j * n + e];
            reinterpret_cast<V*>(p)[j] = v;
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) p[j] = x[j];
    }
}

// One sub-panel (W columns of the current window) factored in LDS.
//
// Thread t owns rows i = t (mod PT) of the sub-panel for the whole call, so
// the per-column passes (pivot swap, reflector dot products, rank-1 update)
// touch only the owner's rows and need no barrier between them; the two
// block sums per column carry everything shared: the trailing norms together
// with row c of every column (which gives the pivot's leading entry), then
// the dot products of the reflector with every column.  The norms for the
// next column are accumulated during the update.  Thread t < W owns row t of
// the compact-WY factor, thread 0 the local pivot order.
template <typename T, int W>
__global__ void __launch_bounds__(PT) qr_panel_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                      int* __restrict__ iaux, T* __restrict__ ws,
                                                      const QRProblemDev* __restrict__ probs,
                                                      const int* __restrict__ plist, int sub) {
    constexpr int S = panel_stride<T, W>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* P = reinterpret_cast<T*>(smem_raw);
    const QRProblemDev q = probs[plist[blockIdx.x]];
    Aux<T> X(aux, iaux, ws, q);
    const int t = threadIdx.x;
    __shared__ __align__(16) T red[2 * W * (PT / 64 + 1)];
    __shared__ T rowc[W];     // row c of the sub-panel, published by its owner
    __shared__ T Tfs[W][W + 1];
    __shared__ int lperm[W];
    __shared__ int gperm_old[W];
    if (X.state[1] || X.state[0] >= 0) {
        if (t == 0) X.state[4] = 0;
        return;
    }
    const int J0 = X.state[2], WO = X.state[3];
    const int j0 = J0 + sub * W;
    if (sub * W >= WO) {
        if (t == 0) X.state[4] = 0;
        return;
    }
    const int nbe = min(W, WO - sub * W);
    const int pr = q.p - j0;
    T* Ab = A + q.offA + (int64_t)j0 * q.p + j0;    // sub-panel origin
    // load (columns past nbe zero-filled); first norms and row 0 on the fly
    T nr[W];   // trailing norms^2 of the columns (rows >= c)
#pragma unroll
    for (int j = 0; j < W; ++j) nr[j] = T(0);
    for (int i = t; i < pr; i += PT) {
        T x[W];
#pragma unroll
        for (int j = 0; j < W; ++j) x[j] = j < nbe ? Ab[(int64_t)j * q.p + i] : T(0);
        store_row<T, W>(P + i * S, x);
#pragma unroll
        for (int j = 0; j < W; ++j) nr[j] += x[j] * x[j];
        if (i == 0)
#pragma unroll
            for (int j = 0; j < W; ++j) rowc[j] = x[j];
    }
    if (t < W) {
#pragma unroll
        for (int j = 0; j < W; ++j) Tfs[t][j] = T(0);
    }
    if (t == 0)
        for (int j = 0; j < W; ++j) lperm[j] = j;
    int parity = 0;
    int nref = nbe;
    const T r11 = X.r11[0];
    // columns unrolled (static_for): every column index below is a
    // compile-time constant; a truncation stops the remaining columns
    bool stop = false;
    static_for<0, W>([&](auto C) {
        constexpr int c = decltype(C)::value;
        if (stop || c >= nbe) return;
        block_sum_n<T, W, W * (PT / 64 + 1)>(nr, red, parity);
        int pv = c;
        T pn = T(-1);
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j >= c && j < nbe && nr[j] > pn) { pn = nr[j]; pv = j; }
        const T x0 = rowc[pv];   // the pivot column's entry in row c
        if (pv != c) {
            for (int i = t; i < pr; i += PT) {
                const T a = P[i * S + c], b = P[i * S + pv];
                P[i * S + c] = b;
                P[i * S + pv] = a;
            }
            if (t == 0) { const int y = lperm[c]; lperm[c] = lperm[pv]; lperm[pv] = y; }
        }
        const T normx = sqrt(pn);
        if (!(normx > T(q.ttol) * r11)) { nref = c; stop = true; return; }
        const T beta = x0 >= T(0) ? -normx : normx;
        const T tau = (beta - x0) / beta;
        const T scl = T(1) / (x0 - beta);
        // d_j = v^T P_j over rows >= c (for j < c: the earlier reflectors);
        // the owner of row c (where v is 1) peels it off
        T d[W];
        int ib = t >= c ? t : t + ((c - t + PT - 1) / PT) * PT;   // first owned row >= c
        const bool own_c = ib == c;
        {
            T x[W];
            if (own_c) load_row<T, W>(P + c * S, x);
#pragma unroll
            for (int j = 0; j < W; ++j) d[j] = own_c ? x[j] : T(0);
        }
        for (int i = own_c ? ib + PT : ib; i < pr; i += PT) {
            T x[W];
            load_row<T, W>(P + i * S, x);
            const T vc = P[i * S + c] * scl;
#pragma unroll
            for (int j = 0; j < W; ++j) d[j] += vc * x[j];
        }
        block_sum_n<T, W, W * (PT / 64 + 1)>(d, red, parity);
        // compact-WY factor column c: T[:c, c] = -tau T[:c, :c] (V[:, :c]^T v_c)
        if (t <= c && t < W) {
            T s2 = T(0);
#pragma unroll
            for (int l = 0; l < W; ++l)
                if (l < c) s2 += Tfs[t][l] * d[l];
            Tfs[t][c] = (t < c) ? -tau * s2 : tau;
        }
        T cf[W];
#pragma unroll
        for (int j = 0; j < W; ++j) cf[j] = (j > c) ? tau * d[j] : T(0);
#pragma unroll
        for (int j = 0; j < W; ++j) nr[j] = T(0);
        if (own_c) {
            T x[W];
            load_row<T, W>(P + c * S, x);
#pragma unroll
            for (int j = 0; j < W; ++j) x[j] -= cf[j];
            store_row<T, W>(P + c * S, x);
            P[c * S + c] = beta;
        }
        for (int i = own_c ? ib + PT : ib; i < pr; i += PT) {
            T x[W];
            load_row<T, W>(P + i * S, x);
            const T vc = P[i * S + c] * scl;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                x[j] -= cf[j] * vc;
                nr[j] += x[j] * x[j];
            }
            store_row<T, W>(P + i * S, x);
            P[i * S + c] = vc;
            if (i == c + 1)
#pragma unroll
                for (int j = 0; j < W; ++j) rowc[j] = x[j];
        }
    });
    // write back (owned rows): R and reflectors to A, reflectors (unit lower) to V
    T* Vb = X.V + (int64_t)(sub * W) * q.p + j0;
    for (int i = t; i < pr; i += PT) {
        T x[W];
        load_row<T, W>(P + i * S, x);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if (j < nbe) {
                Ab[(int64_t)j * q.p + i] = x[j];
                if (j < nref) Vb[(int64_t)j * q.p + i] = (i == j) ? T(1) : (i > j ? x[j] : T(0));
            }
        }
    }
    if (t < nbe) gperm_old[t] = X.perm[j0 + t];
    __syncthreads();
    // rows above the sub-panel hold earlier R entries of these columns: all of
    // them are staged in the (now free) LDS of the sub-panel, then written back
    // in pivot order; nothing to do when the order did not change
    bool moved = false;
    for (int j = 0; j < W; ++j) moved |= lperm[j] != j;
    if (moved && j0 > 0) {
        T* Ac = A + q.offA + (int64_t)j0 * q.p;
        T* Q = P;   // [W][j0]: j0 * W < p * S, within the allocation
        for (int e = t; e < j0 * nbe; e += PT) {
            const int j = e / j0, i = e - j * j0;
            Q[e] = Ac[i + (int64_t)j * q.p];
        }
        __syncthreads();
        for (int e = t; e < j0 * nbe; e += PT) {
            const int j = e / j0, i = e - j * j0;
            Ac[i + (int64_t)j * q.p] = Q[lperm[j] * j0 + i];
        }
    }
    if (t < nbe) X.perm[j0 + t] = gperm_old[lperm[t]];
    for (int e = t; e < NB * NB; e += PT) {
        const int i = e % NB, j = e / NB;
        X.Tf[e] = (i < nref && j < nref && i < W && j < W) ? Tfs[i < W ? i : 0][j < W ? j : 0] : T(0);
    }
    if (t < nref) X.tau[j0 + t] = Tfs[t][t];
    if (t == 0) {
        X.state[4] = nref;
        X.state[6] = j0;
        X.state[7] = nbe;
        if (nref < nbe) X.state[0] = j0 + nref;
        else if (j0 + nbe >= q.k) X.state[0] = q.k;
    }
}

// Apply the sub-panel's reflectors to the remaining columns of the window:
// one workgroup per column, its four waves splitting the rows.
template <typename T, int W>
__global__ void __launch_bounds__(256) qr_inner_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                        int* __restrict__ iaux, T* __restrict__ ws,
                                                        const QRProblemDev* __restrict__ probs,
                                                        const int* __restrict__ plist, int sub) {
    const QRProblemDev q = probs[plist[blockIdx.y]];
    Aux<T> X(aux, iaux, ws, q);
    if (X.state[1]) return;
    const int nref = X.state[4];
    if (nref == 0) return;
    const int j0 = X.state[6], nbe = X.state[7];
    const int J0 = X.state[2], WO = X.state[3];
    if (j0 != J0 + sub * W) return;
    const int col = j0 + nbe + blockIdx.x;
    if (col >= J0 + WO) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pr = q.p - j0;
    T* a = A + q.offA + (int64_t)col * q.p + j0;
    const T* Vb = X.V + (int64_t)(sub * W) * q.p + j0;
    __shared__ T part[4][W];
    T acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = T(0);
    for (int i = threadIdx.x; i < pr; i += 256) {
        const T x = a[i];
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j < nref) acc[j] += Vb[(int64_t)j * q.p + i] * x;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = wave_sum(acc[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < W; ++j) part[wave][j] = acc[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = part[0][j] + part[1][j] + part[2][j] + part[3][j];
    T w[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T s2 = T(0);
#pragma unroll
        for (int i = 0; i < W; ++i)
            if (i <= j) s2 += X.Tf[i + j * NB] * acc[i];
        w[j] = j < nref ? s2 : T(0);
    }
    for (int i = threadIdx.x; i < pr; i += 256) {
        T x = a[i];
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j < nref) x -= Vb[(int64_t)j * q.p + i] * w[j];
        a[i] = x;
    }
}

// Sum the split-K partials of W = V^T C (trailing columns, fixed order).
template <typename T>
__global__ void __launch_bounds__(256) qr_wsum_kernel(T* __restrict__ aux, int* __restrict__ iaux,
                                                       T* __restrict__ ws,
                                                       const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, ws, q);
    if (X.state[1]) return;
    const int J0 = X.state[2], WO = X.state[3];
    const int n = q.k + q.r;
    const int ncols = WIN + n - (J0 + WO);
    const int nch = (q.p - J0 + QR_RC - 1) / QR_RC;
    const int64_t chunk = (int64_t)WIN * (WIN + n);
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < (int64_t)WIN * ncols;
         e += (int64_t)gridDim.x * 256) {
        T s = T(0);
        for (int c = 0; c < nch; ++c) s += X.Wp[c * chunk + e];
        X.Ws[e] = s;
    }
}

// Window compact-WY factor from the Gram matrix G = V^T V (first WIN columns
// of the reduced W).  Its inverse is upper triangular with 1 / tau_j on the
// diagonal and G above it (Joffrain et al., "Accumulating Householder
// transformations, revisited", 2006), so lane j back-substitutes column j of
// the factor against that matrix, all 64 columns at once; an absent
// reflector (tau = 0) gets a zero row and column.
template <typename T>
__global__ void __launch_bounds__(64) qr_tbuild_kernel(T* __restrict__ aux, int* __restrict__ iaux,
                                                        T* __restrict__ ws,
                                                        const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.x];
    Aux<T> X(aux, iaux, ws, q);
    if (X.state[1]) return;
    const int J0 = X.state[2];
    const int j = threadIdx.x;
    __shared__ __align__(16) T Gc[WIN][WIN];    // Gc[i][l] = G[l][i]
    __shared__ T Tt[WIN][WIN + 1];
    __shared__ T tau_s[WIN];
    for (int i = 0; i < WIN; ++i) Gc[i][j] = X.Ws[j + (int64_t)i * WIN];
    tau_s[j] = (J0 + j < q.k) ? X.tau[J0 + j] : T(0);
    __syncthreads();
    T r[WIN];
#pragma unroll
    for (int l = 0; l < WIN; ++l) r[l] = (l == j) ? T(1) : T(0);
#pragma unroll
    for (int i = WIN - 1; i >= 0; --i) {
        const T x = r[i] * tau_s[i];
        Tt[i][j] = x;
#pragma unroll
        for (int l = 0; l < i; ++l) r[l] -= Gc[i][l] * x;
    }
    __syncthreads();
    for (int c = 0; c < WIN; ++c) X.Tw[j + c * WIN] = Tt[j][c];
}

// Exact trailing norms (rows >= J0 + WO) of the remaining candidates.
template <typename T>
__global__ void __launch_bounds__(256) qr_norms_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                        int* __restrict__ iaux,
                                                        const QRProblemDev* __restrict__ probs) {
    const QRProblemDev q = probs[blockIdx.y];
    Aux<T> X(aux, iaux, nullptr, q);
    if (X.state[1] || X.state[0] >= 0) return;
    const int J0 = X.state[2], WO = X.state[3];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = J0 + WO + blockIdx.x * 4 + wave;
    if (col >= q.k) return;
    const T* a = A + q.offA + (int64_t)col * q.p;
    T s = T(0);
    for (int i = J0 + WO + lane; i < q.p; i += 64) s += a[i] * a[i];
    s = wave_sum(s);
    if (lane == 0) X.norms[col] = s;
}

// R11 X = (Q^T K(Z, X^rs))[0:rank, :], then T[perm[i], :] = X[i, :] with zero
// rows for truncated columns.  Blocked back substitution from the bottom, one
// 64-row block per call: the block's right-hand sides (already updated by the
// blocks below, in place in the K(Z, X^rs) columns) are solved against the
// diagonal block of R staged in LDS, one wave per right-hand side and one
// lane per row, and the solution rows are written both in place (for the
// update of the rows above, a grouped GEMM between calls) and to T through
// the pivot order.  Rows at or past the rank get zeros.
template <typename T>
__global__ void __launch_bounds__(256) qr_trsm_kernel(T* __restrict__ A, T* __restrict__ aux,
                                                       int* __restrict__ iaux, T* __restrict__ Tout,
                                                       T* __restrict__ Tsec,
                                                       const QRProblemDev* __restrict__ probs,
                                                       const int* __restrict__ plist, int step) {
    __shared__ T Rb[64][65];
    const QRProblemDev q = probs[plist[blockIdx.y]];
    Aux<T> X(aux, iaux, nullptr, q);
    const int rank = X.state[0] < 0 ? q.k : X.state[0];
    if (step == 0 && blockIdx.x == 0 && threadIdx.x == 0 && q.rec) q.rec[0] = (double)rank;
    const int nblk = (q.k + 63) / 64;
    const int I = nblk - 1 - step;
    if (I < 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + wave;
    if (blockIdx.x * 4 >= q.r) return;
    const int i0 = I * 64, nb = min(64, q.k - i0);
    const T* Ab = A + q.offA;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        Rb[r][c] = (r < nb && c < nb) ? Ab[(i0 + r) + (int64_t)(i0 + c) * q.p] : T(0);
    }
    __syncthreads();
    if (col >= q.r) return;
    T* xc = A + q.offA + (int64_t)(q.k + col) * q.p + i0;
    T xv = (lane < nb && i0 + lane < rank) ? xc[lane] : T(0);
    const int top = min(nb, rank - i0);       // rows of the block inside the rank
    for (int i = top - 1; i >= 0; --i) {
        const T xi = read_lane(xv, i) / Rb[i][i];
        if (lane < i) xv -= xi * Rb[lane][i];
        if (lane == i) xv = xi;
    }
    if (lane < nb) {
        xc[lane] = xv;
        (q.staged ? Tsec : Tout)[q.offT + X.perm[i0 + lane] + (int64_t)col * q.k] = xv;
    }
}

constexpr size_t LDS_BUDGET = 150 * 1024;

// raise a kernel's dynamic-LDS limit once per process to what the 160 KB of
// a gfx950 CU leaves next to the kernel's static LDS; returns that limit
static size_t allow_lds(const void* fn) {
    static std::mutex mu;
    static std::map<const void*, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(fn);
    if (it != done.end()) return it->second;
    hipFuncAttributes at;
    RSD_HIP(hipFuncGetAttributes(&at, fn));
    const size_t lim = 160 * 1024 - at.sharedSizeBytes;
    RSD_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim));
    done[fn] = lim;
    return lim;
}

}  // namespace

int qr_panel_width(int p, int elem_bytes) {
    const size_t eb = (size_t)elem_bytes;
    if (elem_bytes == 4) {
        if ((size_t)panel_stride<float, 16>() * p * eb <= LDS_BUDGET) return 16;
        if ((size_t)panel_stride<float, 8>() * p * eb <= LDS_BUDGET) return 8;
        if ((size_t)panel_stride<float, 4>() * p * eb <= LDS_BUDGET) return 4;
        if ((size_t)panel_stride<float, 2>() * p * eb <= LDS_BUDGET) return 2;
        if ((size_t)panel_stride<float, 1>() * p * eb <= LDS_BUDGET) return 1;
        return 0;
    }
    if ((size_t)panel_stride<double, 16>() * p * eb <= LDS_BUDGET) return 16;
    if ((size_t)panel_stride<double, 8>() * p * eb <= LDS_BUDGET) return 8;
    if ((size_t)panel_stride<double, 4>() * p * eb <= LDS_BUDGET) return 4;
    if ((size_t)panel_stride<double, 2>() * p * eb <= LDS_BUDGET) return 2;
    if ((size_t)panel_stride<double, 1>() * p * eb <= LDS_BUDGET) return 1;
    return 0;
}

template <typename T>
void launch_qr_init(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int max_k,
                    hipStream_t s) {
    if (n_probs <= 0) return;
    hipLaunchKernelGGL(qr_init_kernel<T>, dim3((max_k + 3) / 4, n_probs), dim3(256), 0, s, A, aux,
                       iaux, probs);
    hipLaunchKernelGGL(qr_r11_kernel<T>, dim3(n_probs), dim3(256), 0, s, aux, iaux, probs);
}

template <typename T>
void launch_qr_damp(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int max_k,
                    hipStream_t s) {
    if (n_probs <= 0 || max_k <= 0) return;
    hipLaunchKernelGGL(qr_damp_kernel<T>, dim3((max_k + 255) / 256, n_probs), dim3(256), 0, s, A, aux, iaux,
                       probs);
}

template <typename T>
void launch_qr_select(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, int n_probs,
                      int outer, int max_k, hipStream_t s) {
    if (n_probs <= 0) return;
    int nsort = 2;
    while (nsort < max_k - outer * WIN) nsort <<= 1;
    const size_t shm = (sizeof(T) + sizeof(int)) * (size_t)nsort;
    if (allow_lds((const void*)qr_select_kernel<T, T>) >= shm) {
        hipLaunchKernelGGL((qr_select_kernel<T, T>), dim3(n_probs), dim3(256), shm, s, A, aux, iaux, ws, probs, outer,
                           nsort);
        return;
    }
    const size_t shm_f = (sizeof(float) + sizeof(int)) * (size_t)nsort;
    if (allow_lds((const void*)qr_select_kernel<T, float>) < shm_f) throw HipError("window selection exceeds LDS");
    hipLaunchKernelGGL((qr_select_kernel<T, float>), dim3(n_probs), dim3(256), shm_f, s, A, aux, iaux, ws, probs,
                       outer, nsort);
}

template <typename T>
void launch_qr_move(T* A, int* iaux, T* ws, const QRProblemDev* probs, int n_probs, int phase,
                    hipStream_t s) {
    if (n_probs <= 0) return;
    hipLaunchKernelGGL(qr_move_kernel<T>, dim3(phase == 0 ? 3 * WIN : 2 * WIN, n_probs), dim3(256), 0, s,
                       A, iaux, ws, probs, phase);
}

template <typename T, int W>
static void panel_launch(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs,
                         const int* plist, int n_list, int sub, int max_p, hipStream_t s) {
    auto kfn = qr_panel_kernel<T, W>;
    const size_t shm = (size_t)max_p * panel_stride<T, W>() * sizeof(T);
    if (allow_lds((const void*)kfn) < shm) throw HipError("interpolation panel exceeds LDS");
    hipLaunchKernelGGL(kfn, dim3(n_list), dim3(PT), shm, s, A, aux, iaux, ws, probs, plist, sub);
}

template <typename T>
void launch_qr_panel(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, const int* plist,
                     int n_list, int nb_class, int max_p, int outer, int sub, hipStream_t s) {
    (void)outer;
    if (n_list <= 0) return;
    if (nb_class == 16) panel_launch<T, 16>(A, aux, iaux, ws, probs, plist, n_list, sub, max_p, s);
    else if (nb_class == 8) panel_launch<T, 8>(A, aux, iaux, ws, probs, plist, n_list, sub, max_p, s);
    else if (nb_class == 4) panel_launch<T, 4>(A, aux, iaux, ws, probs, plist, n_list, sub, max_p, s);
    else if (nb_class == 2) panel_launch<T, 2>(A, aux, iaux, ws, probs, plist, n_list, sub, max_p, s);
    else if (nb_class == 1) panel_launch<T, 1>(A, aux, iaux, ws, probs, plist, n_list, sub, max_p, s);
    else throw HipError("bad panel width");
}

template <typename T>
void launch_qr_inner(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, const int* plist,
                     int n_list, int nb_class, int outer, int sub, hipStream_t s) {
    (void)outer;
    if (n_list <= 0) return;
    const dim3 grid(WIN, n_list);
    if (nb_class == 16) hipLaunchKernelGGL((qr_inner_kernel<T, 16>), grid, dim3(256), 0, s, A, aux, iaux, ws, probs, plist, sub);
    else if (nb_class == 8) hipLaunchKernelGGL((qr_inner_kernel<T, 8>), grid, dim3(256), 0, s, A, aux, iaux, ws, probs, plist, sub);
    else if (nb_class == 4) hipLaunchKernelGGL((qr_inner_kernel<T, 4>), grid, dim3(256), 0, s, A, aux, iaux, ws, probs, plist, sub);
    else if (nb_class == 2) hipLaunchKernelGGL((qr_inner_kernel<T, 2>), grid, dim3(256), 0, s, A, aux, iaux, ws, probs, plist, sub);
    else if (nb_class == 1) hipLaunchKernelGGL((qr_inner_kernel<T, 1>), grid, dim3(256), 0, s, A, aux, iaux, ws, probs, plist, sub);
    else throw HipError("bad panel width");
}

template <typename T>
void launch_qr_wsum(T* aux, int* iaux, T* ws, const QRProblemDev* probs, int n_probs, int outer,
                    int max_n, int max_nch, hipStream_t s) {
    (void)outer; (void)max_nch;
    if (n_probs <= 0) return;
    int blocks = (int)std::min<int64_t>(1024, ((int64_t)WIN * (WIN + max_n) + 255) / 256);
    hipLaunchKernelGGL(qr_wsum_kernel<T>, dim3(std::max(blocks, 1), n_probs), dim3(256), 0, s, aux, iaux, ws, probs);
    hipLaunchKernelGGL(qr_tbuild_kernel<T>, dim3(n_probs), dim3(64), 0, s, aux, iaux, ws, probs);
}

template <typename T>
void launch_qr_norms(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int outer,
                     int max_k, hipStream_t s) {
    (void)outer;
    if (n_probs <= 0) return;
    hipLaunchKernelGGL(qr_norms_kernel<T>, dim3((max_k + 3) / 4, n_probs), dim3(256), 0, s, A, aux, iaux, probs);
}

template <typename T>
void launch_qr_trsm(T* A, T* aux, int* iaux, T* Tout, T* Tsec, const QRProblemDev* probs,
                    const int* plist, int n_probs, int max_r, int step, hipStream_t s) {
    if (n_probs <= 0 || max_r <= 0) return;
    hipLaunchKernelGGL(qr_trsm_kernel<T>, dim3((max_r + 3) / 4, n_probs), dim3(256), 0, s, A, aux,
                       iaux, Tout, Tsec, probs, plist, step);
}

#define INST(T)                                                                                   \
    template void launch_qr_init<T>(T*, T*, int*, const QRProblemDev*, int, int, hipStream_t);     \
    template void launch_qr_damp<T>(T*, T*, int*, const QRProblemDev*, int, int, hipStream_t);     \
    template void launch_qr_select<T>(T*, T*, int*, T*, const QRProblemDev*, int, int, int,        \
                                      hipStream_t);                                               \
    template void launch_qr_move<T>(T*, int*, T*, const QRProblemDev*, int, int, hipStream_t);     \
    template void launch_qr_panel<T>(T*, T*, int*, T*, const QRProblemDev*, const int*, int, int,  \
                                     int, int, int, hipStream_t);                                 \
    template void launch_qr_inner<T>(T*, T*, int*, T*, const QRProblemDev*, const int*, int, int,  \
                                     int, int, hipStream_t);                                      \
    template void launch_qr_wsum<T>(T*, int*, T*, const QRProblemDev*, int, int, int, int,         \
                                    hipStream_t);                                                 \
    template void launch_qr_norms<T>(T*, T*, int*, const QRProblemDev*, int, int, int,             \
                                     hipStream_t);                                                \
    template void launch_qr_trsm<T>(T*, T*, int*, T*, T*, const QRProblemDev*, const int*, int,    \
                                    int, int, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace rsd
