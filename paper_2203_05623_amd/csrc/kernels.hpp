// Device-side data descriptors and kernel launchers of the Sternheimer library.
#pragma once

#include "common.hpp"

namespace sth {

// Geometry of the wave-function sphere on the FFT grid, all on the device.
// Internal coefficient order is stick-major: sticks are lines along grid axis 0
// with fixed (m1, m2), sorted by (m1, m2); inside a stick m0 runs -h..h.
struct GridDev {
  int N = 0;            // grid points per axis
  int npw = 0;          // sphere size
  int nst = 0;          // sticks
  int nrow = 0;         // active i1 rows of a plane (rows holding at least one stick)
  const int* stick_off = nullptr;  // [nst + 1] first sphere element of each stick
  const int* elem_pos = nullptr;   // [npw] stick * N + i0 of each element
  const int* stick_i12 = nullptr;  // [nst] i1 * N + i2 of each stick
  const int* row_list = nullptr;   // [nrow] active i1 rows
  const unsigned long long* rowbits = nullptr;  // [N][2] bit i2 set: (i1, i2) holds a stick
                                                // (filled for N <= 128, the tile forms' grids)
  const int* row_srange = nullptr; // [nrow][2] first and one-past-last stick of each active
                                   // row (the sticks of one row are contiguous)
  unsigned long long rowmask[3] = {0, 0, 0};  // bit i1: row i1 is active (N <= 192)
  const double* kin = nullptr;     // [npw] |G|^2 / 2
  const z64* tw64 = nullptr;       // [N] exp(-2 pi i t / N)
  const z32* tw32 = nullptr;       // [N] same, rounded to FP32
  int plan[2] = {0, 0};            // radix plan of the FFT kernels: [0] FP64, [1] FP32
  int plane_kind[2] = {0, 0};      // plane kernel form (0..kPlaneKinds-1): [0] FP64, [1] FP32
  int zfft_kind[2] = {0, 0};       // z-stick kernel form (0..kZfftKinds-1): [0] FP64, [1] FP32
  void* stage = nullptr;           // strip form: [stage_slots][nrow][N] complex scratch planes
  int stage_slots = 0;             //   (sized for FP64; one per resident workgroup)
};

// A set of vectors addressed through a slot list: vector for list entry c is
// base + slots[c] * stride.
template <typename T>
struct VecSet {
  T* base;
  long long stride;
};

enum ZfwdMode : int {
  ZF_PLAIN = 0,   // out = FFT / N^3
  ZF_SHIFT = 1,   // out = FFT / N^3 + (T(G) - eps_slot) * pin
};

// ---- FFT stages (T = double or float working precision) ----
template <typename T, typename Tin>
void launch_zfft_inv(const GridDev& g, VecSet<const Tin> in, VecSet<cpx<T>> sticks,
                     const int* slots, int ncols, hipStream_t st);
// Potential of list entry c: pot_ptr[slots[c]] if pot_ptr is given, else pot.
template <typename T>
void launch_plane_local(const GridDev& g, VecSet<cpx<T>> sticks, const int* slots, int ncols,
                        const T* pot, const T* const* pot_ptr, hipStream_t st);
template <typename T, typename Tout>
void launch_zfft_fwd(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<Tout> out,
                     const int* slots, int ncols, int mode, VecSet<const Tout> pin,
                     const double* eps_slot, hipStream_t st);
template <typename T>
void launch_plane_to_grid(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<cpx<T>> grid,
                          const int* slots, int ncols, hipStream_t st);
// Delta n_j(r) = coef * sum_v Re[conj(psi_v(r)) dpsi_jv(r)]; the sticks of dpsi_jv
// are at sticks.base + (j * nband + v) * sticks.stride, psi_v(r) at psir + band[v] * N^3.
void launch_drho(const GridDev& g, const z64* sticks, long long stick_stride, int nband,
                 const int* bands, const z64* psir, int npert, double coef, double* drho,
                 hipStream_t st);

// LDS attributes of the plane kernels of grid N (call before any graph capture)
void prepare_fft_kernels(int N);
// Whether plane kernel form `kind` can run on this grid in FP64 (fp32 = false)
// or FP32: the tile forms need N <= kTileMaxN, the compact-row form its active
// rows in one workgroup's LDS.
bool plane_kind_available(const GridDev& g, int kind, bool fp32);
constexpr int kRadixPlansHost = 2;   // radix plans per FFT length (see fft.hpp)
constexpr int kPlaneKinds = 5;       // plane kernels: workgroup, wave, strip, persistent and
                                     // compact-row forms
constexpr int kZfftKinds = 2;        // z-stick kernels: workgroup form, wave form
constexpr int kPlaneStrips = 2;      // plane_kind of the strip form
constexpr int kPlanePersistent = 3;  // plane_kind of the persistent single-pass form
constexpr int kPlaneRows = 4;        // plane_kind of the compact-row form
constexpr int kTileMaxN = 96;        // largest grid whose N x (N + 1) FP64 plane tile fits in LDS
constexpr int kStageSlots = 1024;    // strip-form persistent workgroups (up to four per CU)

// ---- dense contractions on MFMA (FP64) ----
// part[s][c][m] = sum_{k in split s} conj(A[m][k]) * B_c[k]     (A rows of length lda);
// real: only its real part (imaginary part 0), half the MFMA work
void launch_gemm_ah_b(const z64* A, int lda, int M, VecSet<const z64> B, const int* slots,
                      int ncols, int K, int kchunk, z64* part, hipStream_t st,
                      bool real = false);
// C[c][m] = sgn * diag[m] * sum_s part[s][c][m]   (diag may be null -> 1);
// transpose: written as C[m][c] instead (row m = <A_m| . >, a Gram matrix row)
void launch_reduce_parts(const z64* part, int nsplit, int ncols, int M, const double* diag,
                         double sgn, z64* C, hipStream_t st, bool transpose = false);
// Y_c[g] = s0 * Y_c[g] + sum_m A[m][g] C[c][m]; if dot_in, also
// dots[c][tile] = sum_{g in tile} Re(conj(dot_in_c[g]) Y_c[g]) for 64-wide tiles of g.
// real: C is real (its imaginary part is not read), half the MFMA work
void launch_gemm_a_c(const z64* A, int lda, int M, const z64* C, VecSet<z64> Y,
                     const int* slots, int ncols, int K, double s0, VecSet<const z64> dot_in,
                     double* dots, hipStream_t st, bool real = false);
// FP32 variants (W and C in FP32, FP32 MFMA accumulation; B, Y, dots FP64 in memory)
void launch_gemm_ah_b(const z32* A, int lda, int M, VecSet<const z64> B, const int* slots,
                      int ncols, int K, int kchunk, z32* part, hipStream_t st,
                      bool real = false);
void launch_reduce_parts(const z32* part, int nsplit, int ncols, int M, const double* diag,
                         double sgn, z32* C, hipStream_t st, bool transpose = false);
void launch_gemm_a_c(const z32* A, int lda, int M, const z32* C, VecSet<z64> Y,
                     const int* slots, int ncols, int K, double s0, VecSet<const z64> dot_in,
                     double* dots, hipStream_t st, bool real = false);
void launch_z64_to_z32(const z64* src, z32* dst, long long n, hipStream_t st);
inline int gemm_a_c_tiles(int K) { return (K + 63) / 64; }

// BF16 variants for the inner operator of STH_MIXED_BF16 solves: W held as two
// bf16 planes (hi, lo) of rows padded to ldw complex, products
// a_lo b_hi + a_hi b_lo + a_hi b_hi with FP32 accumulation (k_gemm_bf16.hip)
struct bz {
  __bf16 x, y;
};
// row pitch of the bf16 planes: a multiple of 64 with a full LDS stage of slack
inline int bf16_ldw(int K) { return ((K + 63) / 64) * 64 + 64; }
void launch_split_w(const z32* W, int M, int K, int ldw, bz* Wb, hipStream_t st);
// Wb: the hi plane of the rows used; the lo plane starts wplane elements later.
// The product runs over the K columns from column koff of those rows (koff a
// multiple of 4, koff + max(K rounded up to 64, K + 31) <= ldw: the reads of
// the last tiles stay in the row); B and Y are given at that column.
// scratch (scratch_bytes): device memory free for the call, where the vectors
// (2 ncols ldw bz) or C (2 ncols Mp bz, Mp = M rounded up to 32) are split
// into bf16 hi/lo planes once before the product.
void launch_gemm_ah_b_bf16(const bz* Wb, long long wplane, int ldw, int koff, int M,
                           VecSet<const z64> B, const int* slots, int ncols, int K, int kchunk,
                           z32* part, bz* scratch, size_t scratch_bytes, hipStream_t st);
void launch_gemm_a_c_bf16(const bz* Wb, long long wplane, int ldw, int koff, int M, const z32* C,
                          VecSet<z64> Y, const int* slots, int ncols, int K, double s0,
                          VecSet<const z64> dot_in, double* dots, bz* scratch,
                          size_t scratch_bytes, hipStream_t st);

// ---- Gamma-point half-sphere projector products (k_gamma.hip) ----
// C[c][m] = sgn d_m (2 Re sum_s part[s][c][m] - Re(conj(W[m][k0]) X_c[k0])
//                    - 2 Re sum_{kh <= k < k0} conj(W[m][k]) X_c[k]), imaginary part 0:
// the partial sums cover the columns from kh <= k0 on (an aligned start takes
// up to three mirrored columns before G = 0, counted twice by the 2 Re)
template <typename T, typename TW>
void launch_reduce_parts_gamma(const cpx<T>* part, int nsplit, int ncols, int M,
                               const double* diag, double sgn, cpx<T>* C, const TW* W, int ldw,
                               int k0, int kh, VecSet<const z64> X, const int* slots,
                               hipStream_t st);
// Y[mirror[i]] = conj(Y[k0 + 1 + i]), i < nmir, and Im Y[k0] = 0 on the listed vectors
void launch_mirror(VecSet<z64> Y, const int* slots, int ncols, int k0, int nmir,
                   const int* mirror, hipStream_t st);
// dots[c][t]: Re <a_c, b_c> over the 64-element tile t of the sphere (ntile tiles)
void launch_dots_tiles(VecSet<const z64> a, VecSet<const z64> b, const int* slots, int ncols,
                       int npw, int ntile, double* dots, hipStream_t st);
// out[r]: largest |W_r(-G) - conj W_r(G)| over the half sphere; out[R + r]: largest |W_r|
void launch_sym_check(const z64* W, int R, int npw, int k0, int nmir, const int* mirror,
                      double* out, hipStream_t st);

// ---- CG vector kernels (FP64) ----
struct SlotState {
  double* rho;       // [nslots] <r, K r>
  double* bnorm2;    // [nslots] ||b||^2
  double* rnorm2;    // [nslots] ||r||^2 (last)
  double* alpha;     // [nslots]
  double* beta;      // [nslots]
  double* eps;       // [nslots] eps_v of the slot's band
  double* ekin;      // [nslots] kinetic energy of the slot's band (preconditioner)
  double* tol;       // [nslots] relative residual target of the slot's solve
  double* tgt2;      // [nslots] ||r||^2 at which the recurrence stops for a true-residual check
  int* status;       // [nslots] SLOT_*
  int* iters;        // [nslots]
  int* maxit;        // [nslots]
  int* prec;         // [nslots] 0 FP64 operator, 1 FP32 inner operator (defect correction)
};
// Inner target of a mixed-precision solve relative to the residual it starts from:
// the FP32 operator is accurate to ~1e-6 relative, so each inner run reduces the
// true residual by at most this much before the FP64 residual is recomputed.
constexpr double MIXED_INNER_REDUCTION = 1e-5;
enum SlotStatus : int {
  SLOT_FREE = 0,
  SLOT_ACTIVE = 1,
  SLOT_CHECK = 2,       // recursive residual below tol: true residual pending
  SLOT_DONE = 3,
  SLOT_MAXIT = 4,
  SLOT_BREAKDOWN = 5,
  SLOT_NAN = 6,
};
inline int cg_chunks(int npw) { return (npw + 1023) / 1024; }

// r = b, x = 0, p = K b; partials of <b, K b> and ||b||^2
void launch_cg_init(const GridDev& g, VecSet<const z64> b, VecSet<z64> x, VecSet<z64> r,
                    VecSet<z64> p, const int* slots, int ncols, const double* ekin,
                    double* part2, hipStream_t st);
// rho = sum part[0], bnorm2 = sum part[1]; status ACTIVE (or DONE if b == 0)
void launch_cg_init_scalars(const double* part2, int nchunk, const int* slots, int ncols,
                            SlotState s, hipStream_t st);
// alpha = rho / sum(dots); breakdown when <p, A p> <= 0
void launch_cg_alpha(const double* dots, int ntile, const int* slots, int ncols, SlotState s,
                     hipStream_t st);
// x += alpha p; r -= alpha q; partials of <r, K r>, ||r||^2
void launch_cg_update_xr(const GridDev& g, VecSet<z64> x, VecSet<z64> r, VecSet<const z64> p,
                         VecSet<const z64> q, const int* slots, int ncols, SlotState s,
                         double* part2, hipStream_t st);
// beta, rho, convergence test ||r||^2 <= tol^2 ||b||^2, iteration count, maxit
void launch_cg_beta(const double* part2, int nchunk, const int* slots, int ncols, SlotState s,
                    hipStream_t st);
// p = K r + beta p
void launch_cg_update_p(const GridDev& g, VecSet<const z64> r, VecSet<z64> p, const int* slots,
                        int ncols, SlotState s, hipStream_t st);
// r = b - q (true residual) and partial ||r||^2 (part2 layout as above; <r,Kr> too)
void launch_cg_true_resid(const GridDev& g, VecSet<const z64> b, VecSet<const z64> q,
                          VecSet<z64> r, const int* slots, int ncols, const double* ekin_slot,
                          double* part2, hipStream_t st);
// after a true residual: DONE if ||r|| <= tol ||b||, else restart (rho = <r, K r>, beta = 0);
// final_only: only store the true ||r||^2 of a slot that has already stopped
void launch_cg_check_true(const double* part2, int nchunk, const int* slots, int ncols,
                          SlotState s, hipStream_t st, bool final_only = false);

// ---- small helpers ----
void launch_copy_vecs(VecSet<const z64> src, VecSet<z64> dst, const int* slots_src,
                      const int* slots_dst, int ncols, int n, hipStream_t st);
void launch_scale_vecs(VecSet<z64> v, const int* slots, int ncols, int n, double s,
                       hipStream_t st);
void launch_permute_in(const z64* src, long long sstride, z64* dst, long long dstride,
                       const int* perm, int n, int ncols, hipStream_t st);
void launch_permute_out(const z64* src, long long sstride, z64* dst, long long dstride,
                        const int* perm, int n, int ncols, hipStream_t st);
void launch_to_f32(const double* src, float* dst, long long n, hipStream_t st);

// ---- block operations of the valence solver (vectors contiguous, stride n) ----
// out[i] = ||v_i||^2 for i < nvec
void launch_row_norms(const z64* v, int nvec, int n, double* out, hipStream_t st);
// v_i *= f[i]
void launch_scale_rows(z64* v, int nvec, int n, const double* f, hipStream_t st);
// R_i = HX_i - theta_i X_i, W_i = R_i / (max(T - theta_i, 0) + 1), out[i] = ||R_i||^2
void launch_resid_precond(const GridDev& g, const z64* X, const z64* HX, const double* theta,
                          int nvec, z64* W, double* out, hipStream_t st);
// C[c][m] = U[(m0 + m) * ldu + col0 + c] * (scale ? scale[col0 + c] : 1), c < nc, m < nm
void launch_cols_to_rows(const z64* U, int ldu, int m0, int nm, int col0, int nc,
                         const double* scale, z64* C, hipStream_t st);

// ---- dielectric eigensolver (real grid functions, stride ld between vectors) ----
// LDS attributes of the full-grid FFT kernels of grid N (N <= kTileMaxN)
void prepare_grid_fft(int N);
// in-place full-grid 3D FFT of ncols grids: sign -1 forward, +1 inverse, unnormalised
void launch_grid_fft(int N, int plan, int sign, z64* data, long long stride, int ncols,
                     const z64* tw, hipStream_t st);
// coefficients *= scale (sqrt(4 pi) / |G|)^power inside 0 < |m|^2 <= m2max, 0 elsewhere
void launch_coulomb_filter(z64* data, long long stride, int ncols, int N, int m2max, double b,
                           int power, double scale, hipStream_t st);
void launch_real_to_z(const double* in, long long istride, z64* out, long long ostride,
                      long long n, int ncols, hipStream_t st);
void launch_z_to_real(const z64* in, long long istride, double* out, long long ostride,
                      long long n, int ncols, hipStream_t st);
// C[i][j] = w <A_i, B_j> for i < na, j < nb
void launch_gram(const double* A, long long lda, int na, const double* B, long long ldb, int nb,
                 long long n, double w, double* C, hipStream_t st);
// Y_j = beta Y_j + sum_{i < m} X_i C[i][j] for j < k (Y must not alias X)
void launch_combine(const double* X, long long ldx, int m, const double* C, int k, long long n,
                    double beta, double* Y, long long ldy, hipStream_t st);
// R_j = AY_j - lam_j Y_j for j < k (lam on the device)
void launch_ritz_resid(const double* AY, const double* Y, long long ld, const double* lam, int k,
                       long long n, double* R, hipStream_t st);
void launch_scale_vec(double* x, long long n, double s, hipStream_t st);

// ---- Lanczos chains (complex vectors of length n; chain vector (k, m) at
// X + k xs_k + m xs_m) ----
// out[m * ldo + k] = <X_{k,m}|Y_m> for k < nk, m < nm
void launch_chain_dots(const z64* X, long long xs_k, long long xs_m, int nk, const z64* Y,
                       long long ys_m, int nm, int n, z64* out, int ldo, hipStream_t st);
// r_m = Hq_m - Re(alpha_m) q_m - beta_m qprev_m (qprev may be null)
void launch_lanczos_three_term(const z64* Hq, const z64* q, const z64* qprev, const z64* alpha,
                               const double* beta, int nm, int n, z64* r, hipStream_t st);
// r_m -= sum_{k < l} c[m * ldc + k] Q_{k,m}   (Q vectors contiguous: (k nm + m) n)
void launch_chain_orth(const z64* Q, int nm, int n, const z64* c, int ldc, int l, z64* r,
                       hipStream_t st);
// out_m = in_m / s[m]
void launch_chain_div(const z64* in, const double* s, int nm, int n, z64* out, hipStream_t st);
// out = a A + b B + c C over n complex elements (C may be null; out may alias C)
void launch_block_axpbypcz(long long n, double a, const z64* A, double b, const z64* B, double c,
                           const z64* C, z64* out, hipStream_t st);

}  // namespace sth
