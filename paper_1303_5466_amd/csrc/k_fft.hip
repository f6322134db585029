// Fast exact float64 product y = A x for the Nystrom matrix on the grid,
// used for the residuals of iterative refinement (Sec. 5, general
// formulation: A = diag(d) + S K S with S = diag(sqrt b) or I).
//
// The off-diagonal part is a two-level Toeplitz matrix in the grid offsets,
// so it is embedded in an Mx x My circulant (powers of two, Mx >= 2 nx,
// My >= 2 ny) and applied through 2-D FFTs: conv = IFFT(C^ . FFT(S x)).  The
// kernel is even in both offsets, so for the real (Laplace) kernel the
// spectrum C^ is real and two right-hand sides travel together as the real
// and imaginary parts of one complex field; for the complex Helmholtz kernel
// (Sec. 5.3) the spectrum is complex (the transforms of its real and
// imaginary parts, each real) and each complex right-hand side (interleaved)
// is one field.  The 1-D transforms are radix-2 in LDS: a workgroup loads
// up to 8 lines (rows, or 8 adjacent columns so that loads stay coalesced)
// in bit-reversed order, runs log2 L butterfly stages in place with one
// barrier each, and writes them back.
#include <mutex>

#include "common.hpp"

namespace rsd {

namespace {

constexpr double INV_2PI = 0.15915494309189533576888376337251;
constexpr size_t FFT_LDS = 144 * 1024;

__device__ inline unsigned bitrev(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

__global__ void __launch_bounds__(256) fft_lines_kernel(double2* __restrict__ data, int L, int logL,
                                                         int64_t nlines, int64_t line_stride,
                                                         int64_t elem_stride, int lpw, int sign) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2* tw = reinterpret_cast<double2*>(smem_raw);   // L / 2 twiddles
    double2* buf = tw + L / 2;                             // lpw lines of L
    const int t = threadIdx.x;
    const int64_t l0 = (int64_t)blockIdx.x * lpw;
    const int nl = (int)min((int64_t)lpw, nlines - l0);
    for (int k = t; k < L / 2; k += 256) {
        double s, c;
        sincospi(2.0 * (double)k / (double)L, &s, &c);
        tw[k] = make_double2(c, sign * s);
    }
    // line-fastest index so that adjacent lines (columns) load adjacent words
    for (int e = t; e < nl * L; e += 256) {
        const int l = e % nl, i = e / nl;
        buf[l * L + bitrev((unsigned)i, logL)] = data[(l0 + l) * line_stride + (int64_t)i * elem_stride];
    }
    __syncthreads();
    for (int s = 1; s <= logL; ++s) {
        const int half = 1 << (s - 1);
        const int tstep = L >> s;          // twiddle stride for this stage
        for (int e = t; e < nl * (L / 2); e += 256) {
            const int l = e / (L / 2), b = e % (L / 2);
            const int grp = b / half, k = b % half;
            const int i0 = grp * 2 * half + k, i1 = i0 + half;
            const double2 w = tw[k * tstep];
            double2* line = buf + l * L;
            const double2 u = line[i0], v = line[i1];
            const double2 wv = make_double2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
            line[i0] = make_double2(u.x + wv.x, u.y + wv.y);
            line[i1] = make_double2(u.x - wv.x, u.y - wv.y);
        }
        __syncthreads();
    }
    for (int e = t; e < nl * L; e += 256) {
        const int l = e % nl, i = e / nl;
        data[(l0 + l) * line_stride + (int64_t)i * elem_stride] = buf[l * L + i];
    }
}

// C[u][v] = K offset table at (|du|, |dv|) with du = u or u - Mx (both within
// the grid), zero elsewhere and at the origin (the diagonal is separate).
__global__ void circulant_kernel(double2* __restrict__ C, int64_t nx, int64_t ny, int Mx, int My,
                                 KernelDesc kd) {
    const int64_t n = (int64_t)Mx * My;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t u = e / My, v = e % My;
        const int64_t du = u < nx ? u : (Mx - u < nx ? Mx - u : -1);
        const int64_t dv = v < ny ? v : (My - v < ny ? My - v : -1);
        double re = 0.0, im = 0.0;
        if (du >= 0 && dv >= 0 && (du | dv) != 0) {
            const double rho2 = (double)(du * du + dv * dv);
            if (kd.type == 1) {       // (i/4) H0^(1)(k r) = -Y0/4 + i J0/4
                const double z = kd.k * kd.h * sqrt(rho2);
                re = kd.h * kd.h * (-0.25 * y0(z));
                im = kd.h * kd.h * (0.25 * j0(z));
            } else {
                re = kd.h * kd.h * INV_2PI * (kd.logh + 0.5 * log(rho2));
            }
        }
        C[e] = make_double2(re, im);
    }
}

__global__ void spectrum_kernel(double* __restrict__ Cr, const double2* __restrict__ C, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        Cr[e] = C[e].x;
}

__global__ void spectrum_c_kernel(double2* __restrict__ Cc, const double2* __restrict__ C, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        Cc[e] = C[e];
}

// complex right-hand side c (interleaved, grid order): field = S x_c zero-padded
__global__ void pack_c_kernel(double2* __restrict__ X, const double* __restrict__ x, int64_t N, int c,
                              int64_t nx, int64_t ny, int Mx, int My, KernelDesc kd) {
    const int64_t n = (int64_t)Mx * My;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t u = e / My, v = e % My;
        double re = 0.0, im = 0.0;
        if (u < nx && v < ny) {
            const int64_t g = u * ny + v;
            const double s = kd.has_b ? kd.sb[g] : 1.0;
            re = s * x[2 * (g + (int64_t)c * N)];
            im = s * x[2 * (g + (int64_t)c * N) + 1];
        }
        X[e] = make_double2(re, im);
    }
}

__global__ void mul_c_kernel(double2* __restrict__ X, const double2* __restrict__ Cc, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double2 c = Cc[e], z = X[e];
        X[e] = make_double2(c.x * z.x - c.y * z.y, c.x * z.y + c.y * z.x);
    }
}

// y_c = S conv / (Mx My) + d x_c, d = 1 + b sc (contrast) or a + sc (complex sc)
__global__ void unpack_c_kernel(double* __restrict__ y, const double2* __restrict__ X,
                                const double* __restrict__ x, int64_t N, int c, int64_t nx, int64_t ny,
                                int My, double scale, KernelDesc kd) {
    for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < N; g += (int64_t)gridDim.x * 256) {
        const int64_t i = g / ny, j = g % ny;
        const double2 z = X[i * My + j];
        double s = 1.0, dr, di;
        if (kd.has_b) {
            s = kd.sb[g];
            dr = 1.0 + s * s * kd.sc_re;
            di = s * s * kd.sc_im;
        } else {
            dr = (kd.a ? kd.a[g] : 1.0) + kd.sc_re;
            di = kd.sc_im;
        }
        const int64_t o = 2 * (g + (int64_t)c * N);
        const double xr = x[o], xi = x[o + 1];
        y[o] = s * (z.x * scale) + dr * xr - di * xi;
        y[o + 1] = s * (z.y * scale) + dr * xi + di * xr;
    }
}

// field = (S x_c0) + i (S x_c1) zero-padded (c1 absent when c0 is the last)
__global__ void pack_kernel(double2* __restrict__ X, const double* __restrict__ x, int64_t N,
                            int c0, int nrhs, int64_t nx, int64_t ny, int Mx, int My, KernelDesc kd) {
    const int64_t n = (int64_t)Mx * My;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t u = e / My, v = e % My;
        double re = 0.0, im = 0.0;
        if (u < nx && v < ny) {
            const int64_t g = u * ny + v;
            const double s = kd.has_b ? kd.sb[g] : 1.0;
            re = s * x[g + (int64_t)c0 * N];
            if (c0 + 1 < nrhs) im = s * x[g + (int64_t)(c0 + 1) * N];
        }
        X[e] = make_double2(re, im);
    }
}

__global__ void mul_kernel(double2* __restrict__ X, const double* __restrict__ Cr, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double c = Cr[e];
        const double2 z = X[e];
        X[e] = make_double2(c * z.x, c * z.y);
    }
}

// y = S conv / (Mx My) + d x for the two columns carried by the field
__global__ void unpack_kernel(double* __restrict__ y, const double2* __restrict__ X,
                              const double* __restrict__ x, int64_t N, int c0, int nrhs,
                              int64_t nx, int64_t ny, int My, double scale, KernelDesc kd) {
    for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < N; g += (int64_t)gridDim.x * 256) {
        const int64_t i = g / ny, j = g % ny;
        const double2 z = X[i * My + j];
        double dg, s = 1.0;
        if (kd.has_b) { s = kd.sb[g]; dg = 1.0 + s * s * kd.sc_re; }
        else dg = (kd.a ? kd.a[g] : 1.0) + kd.sc_re;
        y[g + (int64_t)c0 * N] = s * (z.x * scale) + dg * x[g + (int64_t)c0 * N];
        if (c0 + 1 < nrhs) y[g + (int64_t)(c0 + 1) * N] = s * (z.y * scale) + dg * x[g + (int64_t)(c0 + 1) * N];
    }
}

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

void fft2(double2* X, int Mx, int My, int sign, hipStream_t s) {
    static std::once_flag attr;
    std::call_once(attr, [] {
        RSD_HIP(hipFuncSetAttribute((const void*)fft_lines_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)FFT_LDS));
    });
    // rows: My-point transforms, one row after another in memory
    {
        const int L = My;
        const int lpw = (int)std::min<size_t>(8, (FFT_LDS - (size_t)L / 2 * 16) / ((size_t)L * 16));
        const size_t shm = ((size_t)L / 2 + (size_t)lpw * L) * 16;
        hipLaunchKernelGGL(fft_lines_kernel, dim3((unsigned)((Mx + lpw - 1) / lpw)), dim3(256), shm, s,
                           X, L, ilog2(L), (int64_t)Mx, (int64_t)My, (int64_t)1, lpw, sign);
    }
    // columns: Mx-point transforms, 8 adjacent columns per workgroup
    {
        const int L = Mx;
        const int lpw = (int)std::min<size_t>(8, (FFT_LDS - (size_t)L / 2 * 16) / ((size_t)L * 16));
        const size_t shm = ((size_t)L / 2 + (size_t)lpw * L) * 16;
        hipLaunchKernelGGL(fft_lines_kernel, dim3((unsigned)((My + lpw - 1) / lpw)), dim3(256), shm, s,
                           X, L, ilog2(L), (int64_t)My, (int64_t)1, (int64_t)My, lpw, sign);
    }
}

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(4096, (n + 255) / 256); }

}  // namespace

bool fft_matvec_sizes(int64_t nx, int64_t ny, int* Mx, int* My) {
    int a = 1, b = 1;
    while (a < 2 * nx) a <<= 1;
    while (b < 2 * ny) b <<= 1;
    *Mx = a;
    *My = b;
    return a <= 4096 && b <= 4096;
}

void launch_fft_spectrum(double* Cr, double2* work, int64_t nx, int64_t ny, int Mx, int My,
                         KernelDesc kd, hipStream_t s) {
    const int64_t n = (int64_t)Mx * My;
    hipLaunchKernelGGL(circulant_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, nx, ny, Mx, My, kd);
    fft2(work, Mx, My, -1, s);
    if (kd.type == 1)
        hipLaunchKernelGGL(spectrum_c_kernel, dim3(grid_for(n)), dim3(256), 0, s,
                           reinterpret_cast<double2*>(Cr), work, n);
    else
        hipLaunchKernelGGL(spectrum_kernel, dim3(grid_for(n)), dim3(256), 0, s, Cr, work, n);
}

void launch_fft_matvec(double* y, const double* x, int nrhs, const double* Cr, double2* work,
                       int64_t nx, int64_t ny, int Mx, int My, KernelDesc kd, hipStream_t s) {
    const int64_t N = nx * ny, n = (int64_t)Mx * My;
    const double scale = 1.0 / (double)n;
    if (kd.type == 1) {       // complex kernel and vectors: one right-hand side per field
        const double2* Cc = reinterpret_cast<const double2*>(Cr);
        for (int c = 0; c < nrhs; ++c) {
            hipLaunchKernelGGL(pack_c_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, x, N, c, nx, ny, Mx, My, kd);
            fft2(work, Mx, My, -1, s);
            hipLaunchKernelGGL(mul_c_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, Cc, n);
            fft2(work, Mx, My, +1, s);
            hipLaunchKernelGGL(unpack_c_kernel, dim3(grid_for(N)), dim3(256), 0, s, y, work, x, N, c, nx, ny, My, scale, kd);
        }
        return;
    }
    for (int c0 = 0; c0 < nrhs; c0 += 2) {
        hipLaunchKernelGGL(pack_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, x, N, c0, nrhs, nx, ny, Mx, My, kd);
        fft2(work, Mx, My, -1, s);
        hipLaunchKernelGGL(mul_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, Cr, n);
        fft2(work, Mx, My, +1, s);
        hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(N)), dim3(256), 0, s, y, work, x, N, c0, nrhs, nx, ny, My, scale, kd);
    }
}

}  // namespace rsd
