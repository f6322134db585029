// Grouped GEMM on the gfx950 matrix cores (MFMA 16x16x4, f64 or f32).
//
// One launch runs a list of independent products (one per box of a tree
// level, or two per box), each described by a GemmDesc; a flat tile table
// maps workgroups to output tiles, so boxes of different sizes share one
// launch without idle workgroups.  Every per-box dense block update of the
// factorisation (Schur complements, interpolation transforms, the
// Gauss-Jordan rank-nb updates) and the level sweeps of the solve go through
// this kernel.
//
// Work-group: 256 threads = 2 x 2 waves, each wave a (TILE/2)^2 sub-tile of
// 16 x 16 MFMA blocks.  Operand panels (TILE x BK of op(A), BK x TILE of
// op(B)) are staged through double-buffered LDS: the global loads of the
// next panel are in flight while the MFMAs consume the current one, and one
// barrier per panel suffices.  The MFMA is issued with its operands swapped
// (it computes the transposed block), so that a lane's accumulators are
// consecutive rows of one column of C: the epilogue's loads and stores of C
// cover whole column segments.
//
// Split-K: when a launch has too few tiles to occupy the chip, a tile's
// (concatenated) K range is split over `nsplit` work-groups, each of which
// writes its partial tile to a workspace; a second dispatch of the same
// kernel (reduce mode, one work-group per split tile) adds the partials in
// split order, applies alpha / beta and stores C.  The kernel boundary orders
// the two, so no fences or atomics are needed, and the sum does not depend on
// which work-group ran first.
#include "common.hpp"

#include <hip/hip_ext.h>

namespace rsd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// MFMA 16x16x4 (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result element v of lane l is D[r][c]).  Called as step(b, a, acc) it
// returns the transposed product, so C[l % 16][col(l, v)] is element v.
//   f64: D row = l / 16 + 4 v, column = l % 16  ->  col(l, v) = l / 16 + 4 v
//   f32: D row = 4 (l / 16) + v, column = l % 16 ->  col(l, v) = 4 (l / 16) + v
template <> struct Mfma<double> {
    typedef d4 acc_t;
    __device__ static inline int col(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    typedef f4 acc_t;
    __device__ static inline int col(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename T, int TILE>
struct Cfg {
    // k extent of one staged panel (two stages of both operands stay within
    // 64 KB of LDS; 37 KB for the 128-wide tiles)
    static constexpr int BK = (sizeof(T) == 8 && TILE == 128) ? 8 : 16;
    static constexpr int LD = TILE + 16;          // LDS row stride: rows 128 B apart mod 256 B
    static constexpr int NB = TILE / 32;          // 16 x 16 blocks per wave and dimension
    static constexpr int LOADS = TILE * BK / 256; // elements per thread per operand panel
    // Panels are [k][i] in LDS with the low four bits of i XORed by swz(k).
    // Banks hold W words of T per row of the bank array and a panel row
    // starts 16 words further along it, so R consecutive k-rows fill it; the
    // swizzle moves each group of R rows to its own block of W / BK columns.
    // A store whose lanes run along k (BK consecutive k, W / BK columns per
    // group of BK lanes) then touches every bank once, and the MFMA operand
    // reads (R rows x 16 consecutive columns per pass) stay conflict-free:
    // the XOR permutes columns inside their 16-column block.
    static constexpr int W = sizeof(T) == 8 ? 32 : 64;
    static constexpr int R = W / 16;
    __device__ static constexpr int swz(int k) { return (k / R) * (W / BK); }
};

// Loads go through buffer instructions: an element outside the product
// (row or column past M / N, k past K) gets an offset past the descriptor's
// range, for which the hardware returns zero, so the masked loads need no
// branches.  Offsets are 32-bit bytes from a base pointer moved to the tile's
// first row / column (so an operand may exceed 2 GiB); the host keeps what
// one tile reaches from there below RSRC_RANGE, and a masked element's
// offset is RSRC_RANGE itself, the first out-of-range byte.
constexpr int RSRC_RANGE = 0x7ffffff0;
constexpr int OFF_MASKED = RSRC_RANGE;
constexpr int RSRC_WORD3 = 0x00020000;    // raw buffer, 32-bit data format

template <typename T> struct BufLoad;
template <> struct BufLoad<double> {
    __device__ static inline double at(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
};
template <> struct BufLoad<float> {
    __device__ static inline float at(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
};

// Per-thread plan of one operand panel.  Because 256 is a multiple of TILE
// and BK, a thread's elements of a panel share one row (or one k) and step
// through the other index with a constant stride: element q of the thread
// sits q * qs elements after the first (plus ps per panel), is valid while
// r0 + q * rq < rmax and k0 + q * kq < K, and goes to LDS word l[q].
template <typename T, int LOADS>
struct PanelPlan {
    __amdgpu_buffer_rsrc_t rs;
    int off0, qs, ps;
    int r0, rq, rmax, k0, kq;
    int l[LOADS];
};

// op(X) is rows x K (A: rows = M) or K x cols (B): `along_rows` says whether
// memory is contiguous along the tile's row/column index (A without
// transpose, B with transpose) or along k.
template <typename T, int TILE>
using PlanOf = PanelPlan<T, Cfg<T, TILE>::LOADS>;

template <typename T, int TILE>
__device__ inline PlanOf<T, TILE> panel_plan(const T* X, int ld, bool along_rows, int base, int lim) {
    typedef Cfg<T, TILE> C_;
    constexpr int BK = C_::BK, LD = C_::LD;
    const int t = threadIdx.x;
    PlanOf<T, TILE> P;
    // the tile's first row (column) as the descriptor's base
    const T* Xb = along_rows ? X + base : X + (int64_t)base * ld;
    P.rs = __builtin_amdgcn_make_buffer_rsrc((void*)Xb, (short)0, RSRC_RANGE, RSRC_WORD3);
    if (along_rows) {   // element (i = t % TILE, kk = t / TILE + q 256 / TILE)
        const int i = t % TILE, kk = t / TILE;
        P.off0 = i + kk * ld;
        P.qs = (256 / TILE) * ld;
        P.ps = BK * ld;
        P.r0 = base + i; P.rq = 0; P.rmax = lim;
        P.k0 = kk; P.kq = 256 / TILE;
#pragma unroll
        for (int q = 0; q < C_::LOADS; ++q) {
            const int k = kk + q * (256 / TILE);
            P.l[q] = k * LD + (i ^ C_::swz(k));
        }
    } else {            // element (kk = t % BK, i = t / BK + q 256 / BK)
        const int kk = t % BK, i = t / BK;
        P.off0 = kk + i * ld;
        P.qs = (256 / BK) * ld;
        P.ps = BK;
        P.r0 = base + i; P.rq = 256 / BK; P.rmax = lim;
        P.k0 = kk; P.kq = 0;
#pragma unroll
        for (int q = 0; q < C_::LOADS; ++q) P.l[q] = kk * LD + ((i + q * (256 / BK)) ^ C_::swz(kk));
    }
    return P;
}

template <typename T, int TILE>
__device__ inline void load_panel(const PlanOf<T, TILE>& P, int K, int panel, T (&r)[Cfg<T, TILE>::LOADS]) {
    constexpr int BK = Cfg<T, TILE>::BK;
    const int kb = panel * BK;
    const int o = P.off0 + panel * P.ps;
#pragma unroll
    for (int q = 0; q < Cfg<T, TILE>::LOADS; ++q) {
        const bool ok = (P.r0 + q * P.rq < P.rmax) & (kb + P.k0 + q * P.kq < K);
        r[q] = BufLoad<T>::at(P.rs, ok ? (o + q * P.qs) * (int)sizeof(T) : OFF_MASKED);
    }
}

template <typename T, int TILE>
__device__ inline void store_panel(const PlanOf<T, TILE>& P, T* S, const T (&r)[Cfg<T, TILE>::LOADS]) {
#pragma unroll
    for (int q = 0; q < Cfg<T, TILE>::LOADS; ++q) S[P.l[q]] = r[q];
}

// Panels p0 .. p1 - 1 of one K segment, accumulated into acc.
template <typename T, int TILE>
__device__ inline void run_segment(const T* A, int lda, int tA, const T* B, int ldb, int tB, int M,
                                   int N, int K, int row0, int col0, int p0, int p1, T* lds,
                                   typename Mfma<T>::acc_t (&acc)[Cfg<T, TILE>::NB][Cfg<T, TILE>::NB]) {
    typedef Cfg<T, TILE> C_;
    constexpr int LD = C_::LD, NB = C_::NB, BK = C_::BK, PANEL = BK * LD;
    if (p0 >= p1) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * (TILE / 2), wc = (wave & 1) * (TILE / 2);
    const PlanOf<T, TILE> pa = panel_plan<T, TILE>(A, lda, !tA, row0, M);
    const PlanOf<T, TILE> pb = panel_plan<T, TILE>(B, ldb, tB, col0, N);
    // lane part of the MFMA operand reads for each 4-deep k step
    int lo[BK / 4];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        lo[kk / 4] = kr * LD + ((lane & 15) ^ C_::swz(kr));
    }
    T ra[C_::LOADS], rb[C_::LOADS];
    load_panel<T, TILE>(pa, K, p0, ra);
    load_panel<T, TILE>(pb, K, p0, rb);
    __syncthreads();            // the previous segment's last panel is consumed
    store_panel<T, TILE>(pa, lds, ra);
    store_panel<T, TILE>(pb, lds + PANEL, rb);
    __syncthreads();
    // The loop body has no branches (a branch here makes the compiler move
    // the accumulators between register files every panel): the panel after
    // the last one is loaded too (masked to zero past K, unused otherwise) and
    // stored to the idle stage.
    for (int p = p0; p < p1; ++p) {
        const int cur = (p - p0) & 1;
        load_panel<T, TILE>(pa, K, p + 1, ra);
        load_panel<T, TILE>(pb, K, p + 1, rb);
        const T* As = lds + cur * 2 * PANEL;
        const T* Bs = As + PANEL;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[NB], b[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) a[i] = As[lo[kk / 4] + wr + 16 * i];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = Bs[lo[kk / 4] + wc + 16 * j];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[i][j] = Mfma<T>::step(b[j], a[i], acc[i][j]);
        }
        T* Ns = lds + (cur ^ 1) * 2 * PANEL;
        store_panel<T, TILE>(pa, Ns, ra);
        store_panel<T, TILE>(pb, Ns + PANEL, rb);
        __syncthreads();
    }
}

// C element of accumulator (i, j, v) of thread t in a TILE x TILE tile
template <typename T, int TILE>
__device__ inline void tile_coords(int t, int i, int j, int v, int& r, int& c) {
    const int lane = t & 63, wave = t >> 6;
    r = (wave >> 1) * (TILE / 2) + 16 * i + (lane & 15);
    c = (wave & 1) * (TILE / 2) + 16 * j + Mfma<T>::col(lane, v);
}

template <typename T, int TILE>
__device__ inline void store_c(const GemmDesc<T>& d, int gi, int gj, T sum) {
    if (gi < d.M && gj < d.N) {
        T* c = d.C + gi + (int64_t)gj * d.ldc;
        T val = d.alpha * sum;
        const bool zb = gj >= d.zc0 && gj < d.zc1;
        if (d.beta != T(0) && !zb) val += d.beta * *c;
        *c = val;
    }
}

// reduce == 0: tiles[blockIdx.x] is a (split) tile of the product;
// reduce == 1: tiles[blockIdx.x] names a split tile whose partials are summed.
template <typename T, int ROLE, int TILE>
__global__ void __launch_bounds__(256) gemm_kernel(const GemmDesc<T>* __restrict__ descs,
                                                   const TileRef* __restrict__ tiles,
                                                   T* __restrict__ ws, int reduce) {
    typedef Cfg<T, TILE> C_;
    constexpr int NB = C_::NB, BK = C_::BK, PANEL = BK * C_::LD;
    constexpr int PER = NB * NB * 4;               // accumulators per thread
    __shared__ __align__(16) T lds[4 * PANEL];   // two stages of [A | B]
    const TileRef tr = tiles[blockIdx.x];
    const GemmDesc<T> d = descs[tr.desc];
    if (d.guard && *d.guard) return;
    const int row0 = tr.tm * TILE, col0 = tr.tn * TILE;
    const int t = threadIdx.x;
    // partial tiles in thread-major order: accumulator (i, j, v) of thread t
    const T* part = ws + (int64_t)tr.pbase * (PER * 256);

    if (reduce) {
        // split by split (all of a split's loads in flight at once), in order
        T sum[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) sum[e] = T(0);
        for (int sp = 0; sp < tr.nsplit; ++sp) {
            const T* ps = part + (int64_t)sp * (PER * 256) + t;
#pragma unroll
            for (int e = 0; e < PER; ++e) sum[e] += ps[e * 256];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int r, c;
                    tile_coords<T, TILE>(t, i, j, v, r, c);
                    store_c<T, TILE>(d, row0 + r, col0 + c, sum[(i * NB + j) * 4 + v]);
                }
        return;
    }

    const int n1 = d.K > 0 ? (d.K + BK - 1) / BK : 0;
    const int n2 = d.K2 > 0 ? (d.K2 + BK - 1) / BK : 0;
    const int nst = n1 + n2;
    const int st0 = (int)((int64_t)tr.split * nst / tr.nsplit);
    const int st1 = (int)((int64_t)(tr.split + 1) * nst / tr.nsplit);
    typename Mfma<T>::acc_t acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};

    // 64-wide unsplit tiles with beta != 0 load their C tile before the K loop
    // (masked buffer loads: zero outside C or in the beta-zero columns), so
    // that short products do not wait for it afterwards
    constexpr bool PREFETCH = TILE == 64;
    T cpre[PREFETCH ? PER : 1];
    const bool use_pre = PREFETCH && tr.nsplit == 1 && d.beta != T(0);
    if constexpr (PREFETCH) {
        if (use_pre) {
            const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(d.C + row0 + (int64_t)col0 * d.ldc), (short)0, RSRC_RANGE, RSRC_WORD3);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int r, c;
                        tile_coords<T, TILE>(t, i, j, v, r, c);
                        const int gi = row0 + r, gj = col0 + c;
                        const bool ok = (gi < d.M) & (gj < d.N) & !((gj >= d.zc0) & (gj < d.zc1));
                        cpre[(i * NB + j) * 4 + v] =
                            BufLoad<T>::at(rc, ok ? (r + c * d.ldc) * (int)sizeof(T) : OFF_MASKED);
                    }
        }
    }

    // panels [st0, st1) of the concatenated K range: first segment, then second
    run_segment<T, TILE>(d.A, d.lda, d.tA, d.B, d.ldb, d.tB, d.M, d.N, d.K, row0, col0, min(st0, n1),
                         min(st1, n1), lds, acc);
    run_segment<T, TILE>(d.A2, d.lda2, d.tA2, d.B2, d.ldb2, d.tB2, d.M, d.N, d.K2, row0, col0,
                         max(st0, n1) - n1, max(st1, n1) - n1, lds, acc);

    if (tr.nsplit > 1) {
        T* mine = ws + ((int64_t)tr.pbase + tr.split) * (PER * 256);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) mine[((i * NB + j) * 4 + v) * 256 + t] = acc[i][j][v];
        return;
    }
    if constexpr (PREFETCH) {
        if (use_pre) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int r, c;
                        tile_coords<T, TILE>(t, i, j, v, r, c);
                        const int gi = row0 + r, gj = col0 + c;
                        if ((gi < d.M) & (gj < d.N))
                            d.C[gi + (int64_t)gj * d.ldc] =
                                d.alpha * acc[i][j][v] + d.beta * cpre[(i * NB + j) * 4 + v];
                    }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int r, c;
                tile_coords<T, TILE>(t, i, j, v, r, c);
                store_c<T, TILE>(d, row0 + r, col0 + c, acc[i][j][v]);
            }
}

// Products with N <= 16 (the solve's sweeps over a few right-hand sides):
// every A element is used once, so operands go straight from memory to the
// MFMA.  A wave owns one work item -- a 16-row block of C over part `split`
// of `nsplit` of the concatenated K range -- and keeps 8 k-steps of A and B
// loads in flight (masked buffer loads); four independent items per
// work-group, no LDS, no barriers.  Split items write their 16 x 16
// partial to the workspace, and a reduce dispatch (one wave per split block)
// adds the partials in split order.
// Four consecutive elements from a k-contiguous operand (one 16-byte load
// per two doubles or four floats); the whole group is masked at once.
template <typename T> struct BufLoad4;
template <> struct BufLoad4<double> {
    __device__ static inline void at(__amdgpu_buffer_rsrc_t r, int off, double (&x)[4]) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        typedef double dd2 __attribute__((ext_vector_type(2)));
        const u4 lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const u4 hi = __builtin_amdgcn_raw_buffer_load_b128(r, off == OFF_MASKED ? off : off + 16, 0, 0);
        const dd2 a = __builtin_bit_cast(dd2, lo), b = __builtin_bit_cast(dd2, hi);
        x[0] = a[0]; x[1] = a[1]; x[2] = b[0]; x[3] = b[1];
    }
};
template <> struct BufLoad4<float> {
    __device__ static inline void at(__amdgpu_buffer_rsrc_t r, int off, float (&x)[4]) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        typedef float ff4 __attribute__((ext_vector_type(4)));
        const ff4 a = __builtin_bit_cast(ff4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
        x[0] = a[0]; x[1] = a[1]; x[2] = a[2]; x[3] = a[3];
    }
};

// The k order inside a 16-wide chunk is free (it is a sum): lane group
// g = lane / 16 takes k = 4 g + u in MFMA step u, so a lane reads four
// consecutive k of its row -- one vector load when the operand is contiguous
// along k, whole cache lines per instruction either way.
template <typename T>
__device__ inline void skinny_segment(const T* A, int lda, int tA, const T* B, int ldb, int tB, int M,
                                      int N, int ka, int kb, int row0,
                                      typename Mfma<T>::acc_t& acc) {
    if (ka >= kb) return;
    const int lane = threadIdx.x & 63;
    const int row = row0 + (lane & 15), col = lane & 15, g4 = 4 * (lane >> 4);
    const bool rok = row < M, cok = col < N;
    // element offsets: A(row, k) and B(k, col) as (base + (k - ka) * step),
    // from descriptors based at the item's first row and at k = ka
    const int astep = tA ? 1 : lda, bstep = tB ? ldb : 1;
    const int abase = tA ? (lane & 15) * lda : (lane & 15);
    const int bbase = tB ? col : col * ldb;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A + (tA ? (int64_t)row0 * lda : (int64_t)row0) + (int64_t)ka * astep), (short)0, RSRC_RANGE,
        RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc((void*)(B + (int64_t)ka * bstep), (short)0,
                                                                        RSRC_RANGE, RSRC_WORD3);
    constexpr int SZ = (int)sizeof(T);
    kb -= ka;
    int k = 0;
    // whole chunks, two at a time (16 elements in flight per lane)
    for (; k + 32 <= kb; k += 32) {
        T a[2][4], b[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kk = k + 16 * h + g4;
            if (tA) {
                BufLoad4<T>::at(ra, rok ? (abase + kk) * SZ : OFF_MASKED, a[h]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) a[h][u] = BufLoad<T>::at(ra, rok ? (abase + (kk + u) * astep) * SZ : OFF_MASKED);
            }
            if (!tB) {
                BufLoad4<T>::at(rb, cok ? (bbase + kk) * SZ : OFF_MASKED, b[h]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) b[h][u] = BufLoad<T>::at(rb, cok ? (bbase + (kk + u) * bstep) * SZ : OFF_MASKED);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = Mfma<T>::step(b[h][u], a[h][u], acc);
    }
    // the rest, element by element with k masking
    for (; k < kb; k += 16) {
        T a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = k + g4 + u;
            const bool kok = kk < kb;
            a[u] = BufLoad<T>::at(ra, (rok & kok) ? (abase + kk * astep) * SZ : OFF_MASKED);
            b[u] = BufLoad<T>::at(rb, (cok & kok) ? (bbase + kk * bstep) * SZ : OFF_MASKED);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = Mfma<T>::step(b[u], a[u], acc);
    }
}

template <typename T, int ROLE>
__global__ void __launch_bounds__(256) gemm_skinny_kernel(const GemmDesc<T>* __restrict__ descs,
                                                          const TileRef* __restrict__ items, int n_items,
                                                          T* __restrict__ ws, int reduce) {
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= n_items) return;
    const int lane = threadIdx.x & 63;
    const TileRef it = items[item];
    const GemmDesc<T> d = descs[it.desc];
    if (d.guard && *d.guard) return;
    const int row0 = it.tm * 16;
    typename Mfma<T>::acc_t acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
    if (reduce) {
        for (int sp = 0; sp < it.nsplit; ++sp) {
            const T* p = ws + ((int64_t)it.pbase + sp) * 256 + lane;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += p[v * 64];
        }
    } else {
        // K range of this item: k-steps of 4 over the concatenated segments
        const int n1 = (max(d.K, 0) + 3) / 4, n2 = (max(d.K2, 0) + 3) / 4;
        const int s0 = (int)((int64_t)it.split * (n1 + n2) / it.nsplit);
        const int s1 = (int)((int64_t)(it.split + 1) * (n1 + n2) / it.nsplit);
        skinny_segment<T>(d.A, d.lda, d.tA, d.B, d.ldb, d.tB, d.M, d.N, 4 * min(s0, n1),
                          min(4 * min(s1, n1), d.K), row0, acc);
        skinny_segment<T>(d.A2, d.lda2, d.tA2, d.B2, d.ldb2, d.tB2, d.M, d.N, 4 * (max(s0, n1) - n1),
                          min(4 * (max(s1, n1) - n1), max(d.K2, 0)), row0, acc);
        if (it.nsplit > 1) {
            T* p = ws + ((int64_t)it.pbase + it.split) * 256 + lane;
#pragma unroll
            for (int v = 0; v < 4; ++v) p[v * 64] = acc[v];
            return;
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) store_c<T, 16>(d, row0 + (lane & 15), Mfma<T>::col(lane, v), acc[v]);
}

// The solve's products with split K summed inside the work-group: one
// work-group per 16-row item, wave w takes part w of the item's nsplit K
// parts (the partition of gemm_skinny_kernel), the waves' partials meet in
// LDS and wave 0 adds them in part order (0 + p0 + p1 + ..., the order of
// the two-dispatch form) and stores C.  Waves beyond nsplit contribute
// nothing but still pass the barrier.
template <typename T, int ROLE>
__global__ void __launch_bounds__(64 * SKINNY_WG_WAVES) gemm_skinny_wg_kernel(
    const GemmDesc<T>* __restrict__ descs, const TileRef* __restrict__ items) {
    extern __shared__ __align__(16) unsigned char skinny_smem[];
    T* part = reinterpret_cast<T*>(skinny_smem);   // [waves - 1][4][64]
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const TileRef it = items[blockIdx.x];
    const GemmDesc<T> d = descs[it.desc];
    if (d.guard && *d.guard) return;   // the whole work-group (one item)
    const int row0 = it.tm * 16;
    typename Mfma<T>::acc_t acc = typename Mfma<T>::acc_t{0, 0, 0, 0};
    if (w < it.nsplit) {
        const int n1 = (max(d.K, 0) + 3) / 4, n2 = (max(d.K2, 0) + 3) / 4;
        const int s0 = (int)((int64_t)w * (n1 + n2) / it.nsplit);
        const int s1 = (int)((int64_t)(w + 1) * (n1 + n2) / it.nsplit);
        skinny_segment<T>(d.A, d.lda, d.tA, d.B, d.ldb, d.tB, d.M, d.N, 4 * min(s0, n1),
                          min(4 * min(s1, n1), d.K), row0, acc);
        skinny_segment<T>(d.A2, d.lda2, d.tA2, d.B2, d.ldb2, d.tB2, d.M, d.N, 4 * (max(s0, n1) - n1),
                          min(4 * (max(s1, n1) - n1), max(d.K2, 0)), row0, acc);
    }
    if (w > 0 && w < it.nsplit)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[((w - 1) * 4 + v) * 64 + lane] = acc[v];
    __syncthreads();
    if (w != 0) return;
    typename Mfma<T>::acc_t sum = typename Mfma<T>::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) sum[v] += acc[v];
    for (int sp = 1; sp < it.nsplit; ++sp)
#pragma unroll
        for (int v = 0; v < 4; ++v) sum[v] += part[((sp - 1) * 4 + v) * 64 + lane];
#pragma unroll
    for (int v = 0; v < 4; ++v) store_c<T, 16>(d, row0 + (lane & 15), Mfma<T>::col(lane, v), sum[v]);
}

// A launch with optional timing events attached to the dispatch.
template <typename F, typename... Args>
inline void launch_timed_b(F kernel, dim3 grid, dim3 block, size_t shm, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1, Args... args) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
}
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
    launch_timed_b(kernel, grid, dim3(256), 0, s, e0, e1, args...);
}

template <typename T, int ROLE>
void launch_role(const GemmDesc<T>* d, const TileRef* t, int n, int tile, T* ws, int reduce, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1) {
    if (tile == 16) {
        if (reduce < 0) {   // -reduce waves per item, split K summed in the work-group
            const int waves = std::min(-reduce, SKINNY_WG_WAVES);
            launch_timed_b(gemm_skinny_wg_kernel<T, ROLE>, dim3(n), dim3(64 * waves),
                           (size_t)(waves - 1) * 256 * sizeof(T), s, e0, e1, d, t);
            return;
        }
        launch_timed(gemm_skinny_kernel<T, ROLE>, dim3((n + 3) / 4), s, e0, e1, d, t, n, ws, reduce);
        return;
    }
    if (tile == 128)
        launch_timed(gemm_kernel<T, ROLE, 128>, dim3(n), s, e0, e1, d, t, ws, reduce);
    else
        launch_timed(gemm_kernel<T, ROLE, 64>, dim3(n), s, e0, e1, d, t, ws, reduce);
}

}  // namespace

template <typename T>
void launch_gemm(const GemmDesc<T>* d_descs, const TileRef* d_tiles, int n_tiles, int tile, T* ws,
                 int reduce, hipStream_t s, int role, hipEvent_t ev_start, hipEvent_t ev_stop) {
    if (n_tiles <= 0) return;
    switch (role) {
        case 0: launch_role<T, 0>(d_descs, d_tiles, n_tiles, tile, ws, reduce, s, ev_start, ev_stop); break;
        case 1: launch_role<T, 1>(d_descs, d_tiles, n_tiles, tile, ws, reduce, s, ev_start, ev_stop); break;
        case 2: launch_role<T, 2>(d_descs, d_tiles, n_tiles, tile, ws, reduce, s, ev_start, ev_stop); break;
        default: launch_role<T, 3>(d_descs, d_tiles, n_tiles, tile, ws, reduce, s, ev_start, ev_stop); break;
    }
}

template void launch_gemm<double>(const GemmDesc<double>*, const TileRef*, int, int, double*, int,
                                  hipStream_t, int, hipEvent_t, hipEvent_t);
template void launch_gemm<float>(const GemmDesc<float>*, const TileRef*, int, int, float*, int,
                                 hipStream_t, int, hipEvent_t, hipEvent_t);

}  // namespace rsd
