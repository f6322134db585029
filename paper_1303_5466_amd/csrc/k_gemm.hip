// Grouped GEMM on the gfx950 matrix cores (MFMA 16x16x4, f64 or f32).
//
// One launch runs a list of independent products (one per box of a tree
// level, or two per box), each described by a GemmDesc; a flat tile table
// maps workgroups to 64 x 64 output tiles, so boxes of different sizes share
// one launch without idle workgroups.  Every per-box dense block update of
// the factorisation (Schur complements, interpolation transforms, the
// Gauss-Jordan rank-nb updates) and the level sweeps of the solve go through
// this kernel.
#include "common.hpp"

namespace rsd {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Accumulator layout (16 x 16 block, lane l, element v):
//   f64 16x16x4: row = (l / 16) + 4 v,  column = l % 16
//   f32 16x16x4: row = 4 (l / 16) + v,  column = l % 16
// Inputs: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] in both.
template <> struct Mfma<double> {
    typedef d4 acc_t;
    __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static inline acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    typedef f4 acc_t;
    __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static inline acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int TILE = GEMM_TILE;   // 64
constexpr int BK = 16;
constexpr int PAD = 16;
constexpr int LDS_W = TILE + PAD;

template <typename T>
__device__ inline void load_tiles(const T* __restrict__ A, int lda, int tA, const T* __restrict__ B,
                                  int ldb, int tB, int M, int N, int K, int row0, int col0, int k0,
                                  T (&ra)[4], T (&rb)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        int i, kk;
        if (tA == 0) { i = e & 63; kk = e >> 6; }
        else { kk = e & 15; i = e >> 4; }
        const int gi = row0 + i, gk = k0 + kk;
        T v = T(0);
        if (gi < M && gk < K) v = tA == 0 ? A[gi + (int64_t)gk * lda] : A[gk + (int64_t)gi * lda];
        ra[q] = v;
        int j, kb;
        if (tB == 0) { kb = e & 15; j = e >> 4; }
        else { j = e & 63; kb = e >> 6; }
        const int gj = col0 + j, gkb = k0 + kb;
        T w = T(0);
        if (gj < N && gkb < K) w = tB == 0 ? B[gkb + (int64_t)gj * ldb] : B[gj + (int64_t)gkb * ldb];
        rb[q] = w;
    }
}

template <typename T>
__device__ inline void store_tiles(T (*As)[LDS_W], T (*Bs)[LDS_W], int tA, int tB, const T (&ra)[4],
                                   const T (&rb)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + 256 * q;
        int i, kk;
        if (tA == 0) { i = e & 63; kk = e >> 6; }
        else { kk = e & 15; i = e >> 4; }
        As[kk][i] = ra[q];
        int j, kb;
        if (tB == 0) { kb = e & 15; j = e >> 4; }
        else { j = e & 63; kb = e >> 6; }
        Bs[kb][j] = rb[q];
    }
}

template <typename T>
__device__ inline void run_segment(const T* A, int lda, int tA, const T* B, int ldb, int tB, int M,
                                   int N, int K, int row0, int col0, T (*As)[LDS_W],
                                   T (*Bs)[LDS_W], typename Mfma<T>::acc_t (&acc)[2][2]) {
    if (K <= 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    T ra[4], rb[4];
    load_tiles(A, lda, tA, B, ldb, tB, M, N, K, row0, col0, 0, ra, rb);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store_tiles(As, Bs, tA, tB, ra, rb);
        __syncthreads();
        if (k0 + BK < K) load_tiles(A, lda, tA, B, ldb, tB, M, N, K, row0, col0, k0 + BK, ra, rb);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            T a0 = As[kr][wr + (lane & 15)];
            T a1 = As[kr][wr + 16 + (lane & 15)];
            T b0 = Bs[kr][wc + (lane & 15)];
            T b1 = Bs[kr][wc + 16 + (lane & 15)];
            acc[0][0] = Mfma<T>::step(a0, b0, acc[0][0]);
            acc[0][1] = Mfma<T>::step(a0, b1, acc[0][1]);
            acc[1][0] = Mfma<T>::step(a1, b0, acc[1][0]);
            acc[1][1] = Mfma<T>::step(a1, b1, acc[1][1]);
        }
    }
}

// ROLE only names the instantiation (factor levels 0, interpolation 1,
// solve sweeps 2, library calls 3) so that profiles can tell the launch
// sites apart; the code is the same.
template <typename T, int ROLE>
__global__ void __launch_bounds__(256) gemm_kernel(const GemmDesc<T>* __restrict__ descs,
                                                   const TileRef* __restrict__ tiles) {
    __shared__ T As[BK][LDS_W];
    __shared__ T Bs[BK][LDS_W];
    const TileRef tr = tiles[blockIdx.x];
    const GemmDesc<T> d = descs[tr.desc];
    if (d.guard && *d.guard) return;
    const int row0 = tr.tm * TILE, col0 = tr.tn * TILE;
    typename Mfma<T>::acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    run_segment(d.A, d.lda, d.tA, d.B, d.ldb, d.tB, d.M, d.N, d.K, row0, col0, As, Bs, acc);
    run_segment(d.A2, d.lda2, d.tA2, d.B2, d.ldb2, d.tB2, d.M, d.N, d.K2, row0, col0, As, Bs, acc);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = row0 + wr + bi * 16 + Mfma<T>::row(lane, v);
                const int gj = col0 + wc + bj * 16 + (lane & 15);
                if (gi < d.M && gj < d.N) {
                    T* c = d.C + gi + (int64_t)gj * d.ldc;
                    T val = d.alpha * acc[bi][bj][v];
                    const bool zb = gj >= d.zc0 && gj < d.zc1;
                    if (d.beta != T(0) && !zb) val += d.beta * *c;
                    *c = val;
                }
            }
}

}  // namespace

template <typename T>
void launch_gemm(const GemmDesc<T>* d_descs, const TileRef* d_tiles, int n_tiles, hipStream_t s,
                 int role) {
    if (n_tiles <= 0) return;
    switch (role) {
        case 0: hipLaunchKernelGGL((gemm_kernel<T, 0>), dim3(n_tiles), dim3(256), 0, s, d_descs, d_tiles); break;
        case 1: hipLaunchKernelGGL((gemm_kernel<T, 1>), dim3(n_tiles), dim3(256), 0, s, d_descs, d_tiles); break;
        case 2: hipLaunchKernelGGL((gemm_kernel<T, 2>), dim3(n_tiles), dim3(256), 0, s, d_descs, d_tiles); break;
        default: hipLaunchKernelGGL((gemm_kernel<T, 3>), dim3(n_tiles), dim3(256), 0, s, d_descs, d_tiles); break;
    }
}

template void launch_gemm<double>(const GemmDesc<double>*, const TileRef*, int, hipStream_t, int);
template void launch_gemm<float>(const GemmDesc<float>*, const TileRef*, int, hipStream_t, int);

}  // namespace rsd
