// Shared device-side types and launch declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace rsd {

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define RSD_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::rsd::HipError(std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel description passed by value to every generation kernel.
// Off-diagonal entry between grid points p != q:
//   h^2 * K(h * |(du, dv)|) * sb_p * sb_q     (sb = sqrt(b) or 1)
// Diagonal entry of point p:
//   a_p + sc          (no contrast)      or   1 + b_p * sc   (contrast)
// with sc the integral of K over the point's own cell.
//
// Complex kernels (cplx = 1, Helmholtz G = (i/4) H0^(1)(k r)): the factor is
// built for the real symmetric matrix J(M) that carries the complex
// symmetric M = M_re + i M_im on two dofs per point,
//   J(M) = [[M_re, M_im], [M_im, -M_re]],   J(M) [u; w] = [Re g; Im g]
// for M (u - i w) = g; every dof block of a box lists its points twice,
// [sk plane 0; sk plane 1; rs plane 0; rs plane 1] (plane 0 carries the real
// component u, plane 1 carries w = -Im y), so each generated entry is the
// (plane_i, plane_j) component of J of the complex entry.
// ---------------------------------------------------------------------------
struct KernelDesc {
    int type;          // 0 Laplace, 1 Helmholtz
    int has_b;         // contrast present
    double h;          // grid spacing
    double logh;       // log(h)
    double k;          // wavenumber
    double sc_re, sc_im;   // self-cell integral
    const double* a;   // grid-ordered identity coefficient (N) or nullptr
    const double* sb;  // grid-ordered sqrt(b) (N) or nullptr
    int64_t ny;        // grid index g = i * ny + j
    int cplx;          // 1: two dofs per point (J form above)
};

// Plane (0 or 1) of position q of a complex factor's dof block with k
// skeleton and r residual dofs: every point's two dofs are adjacent (plane 0,
// then plane 1), skeleton points first, so the elimination in natural order
// pivots on whole complex entries (a 2 x 2 block [[re, im], [im, -re]] of
// determinant -|z|^2) rather than on real parts alone.
__host__ __device__ inline int dof_plane(int q, int k, int r) {
    (void)k; (void)r;
    return q & 1;
}
// (pi, pj) component of J(re + i im)
__host__ __device__ inline double jform(double re, double im, int pi, int pj) {
    return pi == pj ? (pi ? -re : re) : im;
}

// Per-box record used by the device kernels.
struct BoxDev {
    int x0, y0;
    int k, r;
    int layout;
    int parent;
    int pos;           // which child of the parent
    int child0, child1;
    int level;
    int64_t offF;      // F block offset in the level's arena (elements)
    int64_t offV;      // vector block offset (elements per rhs)
    int64_t offY;      // residual-part block offset (elements per rhs)
};

struct LayoutDev {
    int k, r;
    int off_uv;        // start of the layout's entries in the u/v tables
    int off_inv0, off_inv1;   // start of the inverse maps (child sk -> parent pos)
    int idp;           // interpolation problem (-1 none)
    int64_t offT;      // T block (k x r) in the T arena, -1 if none
};

// Column-major GEMM descriptor: C = alpha * opA(A) * opB(B) + beta * C,
// optionally accumulating a second product opA(A2) * opB(B2) (K2 > 0).
template <typename T>
struct GemmDesc {
    int M, N, K, K2;
    int tA, tB, tA2, tB2;
    const T* A; const T* B; const T* A2; const T* B2;
    T* C;
    int lda, ldb, lda2, ldb2, ldc;
    int zc0, zc1;      // columns [zc0, zc1) of C use beta = 0
    const int* guard;  // if non-null and *guard != 0 the product is skipped
    T alpha, beta;
};

// One work-group of a grouped GEMM launch: output tile (tm, tn) of product
// `desc`, and its part `split` of `nsplit` of the K range; a split tile's
// partials are tiles pbase .. pbase + nsplit - 1 of the workspace.
struct TileRef {
    int desc;
    int tm, tn;
    int split, nsplit, pbase;
};

// Most waves of one work-group of the N <= 16 product kernel with split K
// summed in the work-group (launch_gemm, tile 16, reduce < 0).
constexpr int SKINNY_WG_WAVES = 16;

// Largest byte extent of one GEMM operand from its base pointer (the kernel
// uses 32-bit buffer offsets).
constexpr int64_t GEMM_MAX_OPERAND_BYTES = 0x7ffffff0;

// ------------------------------- launchers ---------------------------------
// tile: 64 or 128 (square output tiles), or 16 for the N <= 16 kernel (one
// 16-row block of C per wave; d_tiles then lists one entry per wave, tm the
// row block); ws: split-K partial tiles;
// reduce: 0 = products (d_tiles: one entry per work-group), 1 = sum the
// partials of the split tiles listed in d_tiles into C; with tile 16, -w =
// one work-group of w waves per 16-row item (d_tiles one entry per item, its
// nsplit K parts summed in the work-group, no partials in ws)
// role: 0 factor levels, 1 interpolation, 2 solve sweeps, 3 library calls
// ev_start / ev_stop (optional): events set to the launch's kernel start
// and end (timing carried by the dispatch, no marker packets)
template <typename T>
void launch_gemm(const GemmDesc<T>* d_descs, const TileRef* d_tiles, int n_tiles, int tile, T* ws,
                 int reduce, hipStream_t s, int role, hipEvent_t ev_start = nullptr,
                 hipEvent_t ev_stop = nullptr);

// generation / assembly
// One factor of a batch group for the merged assembly launches: its arenas
// (F of the level's precision, Fc of the children's) and plan tables.
struct AsmInst {
    void* F;
    const void* Fc;
    const BoxDev* boxes;
    const LayoutDev* layouts;
    const int* lu;
    const int* lv;
    const int* src_c;
    const int* src_i;
    KernelDesc kd;
};
struct GroupItem {
    int inst, box;    // factor of the group, box of that factor
};
template <typename T>
void launch_leaf_F_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_m, hipStream_t s);
template <typename TS, typename TD>
void launch_assemble_F_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_m,
                             hipStream_t s);
template <typename T>
void launch_transpose_group(const AsmInst* insts, const GroupItem* items, int n_items, int max_k, int max_r,
                            hipStream_t s);
template <typename T>
void launch_leaf_F(T* F, const BoxDev* boxes, const int* box_ids, int n_boxes,
                   const LayoutDev* layouts, const int* lu, const int* lv, KernelDesc kd,
                   int max_m, hipStream_t s);
template <typename TS, typename TD>
void launch_assemble_F(TD* F, const TS* Fchild, const BoxDev* boxes, const int* box_ids,
                       int n_boxes, const LayoutDev* layouts, const int* lu, const int* lv,
                       const int* src_c, const int* src_i, KernelDesc kd, int max_m,
                       hipStream_t s);
template <typename T>
void launch_transpose_sr(T* F, const BoxDev* boxes, const int* ids, int n_boxes, int max_k,
                         int max_r, hipStream_t s);
template <typename T>
// geo per problem: ax, ay, sector (-1: plain problem; 0..3: symmetry sector
// ab = a + 2b, entries summed over the reflections of the group with signs
// (-1)^(a gx + b gy)), group (bit 0: u reflection, bit 1: v reflection);
// logh_of: nullptr (every problem uses kd.logh) or log h per problem
void launch_proxy_matrix(T* A, const int64_t* offA, const int* p_of, const int* k_of,
                         const int* r_of, const int* zoff, const int* zu, const int* zv,
                         const int* xoff, const int* xu, const int* xv, const int* geo,
                         const double* logh_of, int n_problems, int max_pn, KernelDesc kd,
                         hipStream_t s);
// T of a box type from solutions kept in a float64 sector arena: the four
// sector solutions of a symmetric type combined, or a plain solution copied,
// converted to the precision of the T arena (see k_gen.hip)
struct SymCombineDesc {
    int64_t offT;      // layout T (k x r, ld k) in the T arena
    int64_t offS;      // sym: sector sc block (k/ns x r/ns, ld k/ns) at offS + sc (k/ns)(r/ns); else k x r
    int k, r;
    int off_sk, off_rs;   // into the orbit / reflection tables (sym only)
    int sym;
    int grp;           // reflection group of a symmetric type (bit 0: u, bit 1: v)
    void* dst;         // nullptr: T at offT in the launch's arena; else the layout's T itself
};
template <typename TS, typename TD>
void launch_sym_combine(TD* Tarena, const TS* Tsec, const SymCombineDesc* d, int n_desc,
                        const int* orb, const int* refl, int max_kr, hipStream_t s);

// QR least squares for T (block column pivoting)
constexpr int QR_NB = 16;     // largest sub-panel width
constexpr int QR_WIN = 64;    // pivoting window / block width of the trailing update
constexpr int QR_RC = 256;    // row chunk of the split-K reflector products
struct QRProblemDev {
    int p, k, r, nb;   // nb: sub-panel width (16, 8, 4, 2 or 1 by the LDS budget)
    int pz;            // rows holding the proxy kernel; rows pz .. p - 1 the damping rows (k or none)
    int sec;           // -1, or the symmetry sector (0..3) this problem solves
    int staged;        // 0: T goes to the T arena; 1: to the staging arena (sector, or another precision)
    int g0, gn;        // sector group: list index of its first problem and number of sectors
                       // (g0 = own index and gn = 1 for a problem solved whole)
    int64_t offA;      // p x (k + r) matrix, ld = p
    int64_t offT;      // output T (k x r), ld = k, in the arena staged selects
    int64_t offAux;    // norms (k), tau (k), sub-panel WY (QR_NB^2), window WY (QR_WIN^2), r11
    int64_t offIaux;   // perm (k), state (8), moves (4 * QR_WIN)
    int64_t offV;      // V workspace p x QR_WIN (unit lower trapezoidal)
    int64_t offTmp;    // column staging for the window permutation, p x 2 QR_WIN
    int64_t offW;      // split-K partials nch x QR_WIN x (QR_WIN + k + r)
    int64_t offWs;     // reduced W, QR_WIN x (QR_WIN + k + r); then W' after the trailing block
    double* rec;       // record of the truncation: kept rank, |R_11| reference, sectors in the group
    double ttol;       // truncation threshold |R_jj| <= ttol |R_11|
    double damp;       // > 0: rows pz + j hold damp |R_11| in column j (damped least squares)
};
template <typename T>
void launch_qr_init(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int max_k,
                    hipStream_t s);
// the damping rows of the problems with damp > 0 (after launch_qr_init)
template <typename T>
void launch_qr_damp(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int max_k,
                    hipStream_t s);
template <typename T>
void launch_qr_select(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, int n_probs,
                      int outer, int max_k, hipStream_t s);
template <typename T>
void launch_qr_move(T* A, int* iaux, T* ws, const QRProblemDev* probs, int n_probs, int phase,
                    hipStream_t s);
// plist: problem ids of one sub-panel width class; the truncation threshold
// is each problem's ttol
template <typename T>
void launch_qr_panel(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, const int* plist,
                     int n_list, int nb_class, int max_p, int outer, int sub, hipStream_t s);
template <typename T>
void launch_qr_inner(T* A, T* aux, int* iaux, T* ws, const QRProblemDev* probs, const int* plist,
                     int n_list, int nb_class, int outer, int sub, hipStream_t s);
template <typename T>
void launch_qr_wsum(T* aux, int* iaux, T* ws, const QRProblemDev* probs, int n_probs, int outer,
                    int max_n, int max_nch, hipStream_t s);
template <typename T>
void launch_qr_norms(T* A, T* aux, int* iaux, const QRProblemDev* probs, int n_probs, int outer,
                     int max_k, hipStream_t s);
int qr_panel_width(int p, int elem_bytes);   // sub-panel width for a p-row problem
template <typename T>
void launch_qr_trsm(T* A, T* aux, int* iaux, T* Tout, T* Tsec, const QRProblemDev* probs,
                    const int* plist, int n_probs, int max_r, int step, hipStream_t s);

// Gauss-Jordan pivot step (see gj kernels)
template <typename T>
struct GJDesc {
    T* X;            // base of the r x ncols block (row 0 = first pivot row)
    int ld;
    int n;           // pivot block size (number of rows)
    int ncols;       // total columns updated
    int pcol;        // column index of the first pivot column
    T* SR;           // nb x ncols side buffer (ld = nb)
    T* SC;           // n x nb side buffer (ld = n)
    int box;         // for error reports
    int* err = nullptr;   // error flag of the block's factor (nullptr: the launch's)
};
template <typename T>
void launch_gj_pivot(const GJDesc<T>* d, int n_desc, int step, int nb, int max_chunks,
                     int* err, int pair, hipStream_t s);

// solve-phase gathers and scatters
template <typename TS, typename TD>
void launch_gather_leaf(TD* V, const TS* f, int64_t ldf, int nrhs, const BoxDev* boxes,
                        const int* box_ids, int n_boxes, const LayoutDev* layouts, const int* lu,
                        const int* lv, const int64_t* perm, int64_t ny, int64_t plane_off, int max_m,
                        hipStream_t s);
template <typename TS, typename TD>
void launch_scatter_leaf(TD* x, int64_t ldx, const TS* V, const TS* Y, int nrhs,
                         const BoxDev* boxes, const int* box_ids, int n_boxes,
                         const LayoutDev* layouts, const int* lu, const int* lv,
                         const int64_t* perm, int64_t ny, int64_t plane_off, int max_m, hipStream_t s);
template <typename TS, typename TD>
void launch_scatter_up(TD* Vparent, const TS* V, int nrhs, const BoxDev* boxes, const int* box_ids,
                       int n_boxes, const LayoutDev* layouts, const int* inv, int max_k,
                       hipStream_t s);
template <typename TS, typename TD>
void launch_gather_down(TD* V, const TS* Vparent, const TS* Yparent, int nrhs,
                        const BoxDev* boxes, const int* box_ids, int n_boxes,
                        const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s);

// exact float64 matvec y = A x on the grid (grid-ordered vectors)
void launch_matvec_table(double* table, int64_t nx, int64_t ny, KernelDesc kd, hipStream_t s);
// FFT form of the exact product (circulant embedding, k_fft.hip); sizes are
// powers of two >= twice the grid sides, false when a side exceeds 4096
bool fft_matvec_sizes(int64_t nx, int64_t ny, int* Mx, int* My);
void launch_fft_spectrum(double* Cr, double2* work, int64_t nx, int64_t ny, int Mx, int My,
                         KernelDesc kd, hipStream_t s);
void launch_fft_matvec(double* y, const double* x, int nrhs, const double* Cr, double2* work,
                       int64_t nx, int64_t ny, int Mx, int My, KernelDesc kd, hipStream_t s);
void launch_matvec(double* y, const double* x, int nrhs, const double* table, int64_t nx,
                   int64_t ny, KernelDesc kd, int cplx, hipStream_t s);

// elementwise helpers
template <typename TS, typename TD>
void launch_convert(TD* dst, const TS* src, int64_t n, hipStream_t s);
void launch_permute(double* dst, const double* src, const int64_t* perm, int64_t n, int nrhs,
                    int width, int to_grid, hipStream_t s);
void launch_axpy_resid(double* r, const double* f, const double* Ax, int64_t n, hipStream_t s);
void launch_add(double* x, const double* d, int64_t n, hipStream_t s);
// compressed forward product (k_hmatvec.hip): charges up, sibling blocks
// across, potentials down, dense leaf blocks; float64 vectors, T in its
// level's precision
template <typename TT>
void launch_hmv_up(const double* X, double* Xpar, const TT* Tarena, int nrhs, const BoxDev* boxes, const int* ids,
                   int n_boxes, const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s);
void launch_hmv_sibling(double* Pot, const double* Xpar, int nrhs, const BoxDev* boxes, const int* ids, int n_boxes,
                        const LayoutDev* layouts, const int* lu, const int* lv, const int* inv, int max_kk,
                        const KernelDesc& kd, hipStream_t s);
template <typename TT>
void launch_hmv_spread(double* Y, const double* Pot, const TT* Tarena, int nrhs, const BoxDev* boxes,
                       const int* ids, int n_boxes, const LayoutDev* layouts, int max_m, hipStream_t s);
void launch_hmv_push(double* Pot, const double* Ypar, int nrhs, const BoxDev* boxes, const int* ids, int n_boxes,
                     const LayoutDev* layouts, const int* inv, int max_k, hipStream_t s);
template <typename TT>
void launch_hmv_leaf(double* y, int64_t ldy, const double* X, const double* Pot, const TT* Tarena, int nrhs,
                     const BoxDev* boxes, const int* ids, int n_boxes, const LayoutDev* layouts, const int* lu,
                     const int* lv, const int64_t* perm, int max_m, const KernelDesc& kd, hipStream_t s);

// squared norms of ncols columns of length n; ws: COLNORM_WS_PER_COL * ncols doubles
constexpr int COLNORM_WS_PER_COL = 128;
void launch_col_norms2(double* out, const double* x, int64_t n, int ncols, double* ws, hipStream_t s);
void launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s);
// contrast scaling and complex plane split / merge around the factored
// system (k_solve.hip)
void launch_scale_split(double* R, const double* f, const double* sb, int64_t N, int nrhs, int cplx,
                        hipStream_t s);
void launch_scale_merge(double* x, const double* X, const double* sb, int64_t N, int nrhs, int cplx,
                        hipStream_t s);

}  // namespace rsd
