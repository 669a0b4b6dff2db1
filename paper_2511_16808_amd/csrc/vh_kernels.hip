// vh_kernels.hip -- gfx950 kernels of the Vanka-smoothed shifted-Laplacian solver.
//
// Every kernel is one sweep over a structured nodal grid, one thread per node
// (or per coarse node / per patch row), linear node index x + nx*(y + ny*z).
// Blocks are remapped so that each XCD owns a contiguous slab of the domain.
// No atomics anywhere: overlap-adds are gathers, reductions run in a fixed order,
// so every result is bitwise reproducible.
#include <type_traits>

#include "vh_launch.h"

namespace vh {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void decode(unsigned i, const Grid& g, int& x, int& y, int& z) {
  grid_decode(i, g, x, y, z);
}
__device__ __forceinline__ bool inside(const Grid& g, int x, int y, int z) {
  return (unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
}
__device__ __forceinline__ long long lin(const Grid& g, int x, int y, int z) {
  return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}
// linear index in the padded layout of the smoother arrays
__device__ __forceinline__ long long linp(const Grid& g, int x, int y, int z) {
  return (long long)x + (long long)g.nxp * ((long long)y + (long long)g.ny * z);
}
__device__ __forceinline__ unsigned node_id() {
  return xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}
static inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define VH_LAUNCH_CHECK()                                 \
  do {                                                    \
    hipError_t e__ = hipGetLastError();                   \
    if (e__ != hipSuccess) return e__;                    \
  } while (0)

// ------------------------------------------------------------------ fill / convert
template <class T>
__global__ __launch_bounds__(256) void k_fill(cpx<T>* __restrict__ p, size_t n, T re, T im) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n; k += stride) p[k] = cmk<T>(re, im);
}

template <class TO, class TI>
__global__ __launch_bounds__(256) void k_convert(const cpx<TI>* __restrict__ a, cpx<TO>* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n; k += stride) b[k] = ccast<TO>(a[k]);
}

hipError_t fill(void* p, size_t n, int prec, double re, double im, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  if (prec == PREC_F64)
    k_fill<double><<<nb, 256, 0, s>>>((cpx<double>*)p, n, re, im);
  else
    k_fill<float><<<nb, 256, 0, s>>>((cpx<float>*)p, n, (float)re, (float)im);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t convert(const void* a, int pa, void* b, int pb, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  if (pa == PREC_F64 && pb == PREC_F32)
    k_convert<float, double><<<nb, 256, 0, s>>>((const cpx<double>*)a, (cpx<float>*)b, n);
  else if (pa == PREC_F32 && pb == PREC_F64)
    k_convert<double, float><<<nb, 256, 0, s>>>((const cpx<float>*)a, (cpx<double>*)b, n);
  else if (pa == PREC_F64)
    k_convert<double, double><<<nb, 256, 0, s>>>((const cpx<double>*)a, (cpx<double>*)b, n);
  else
    k_convert<float, float><<<nb, 256, 0, s>>>((const cpx<float>*)a, (cpx<float>*)b, n);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------ finest operator
// 2nd-order stencil (Sec. 2.1) of eq. (acousitcHelm) with
//   beta = omega^2 kappa^2 - i omega kappa^2 gamma,  gamma = gamma0 + absorbing layer,
//   layer: amp*omega*sum_d ((W - s_d)/W)^2 for s_d < W (s_d = cells to the nearer face),
//   boundary (ABC): ghost node eliminated with du/dn = -i omega kappa u, i.e. the
//   inward neighbour weight doubles and the diagonal gains 2 i omega kappa / h per
//   boundary direction; the row is then scaled by 1/2 per boundary direction
//   (complex-symmetric H).  H_s = H + i alpha omega^2 * scale (eq. (shift), same sign
//   as the attenuation; M = identity of the unscaled rows).
template <int DIM>
__global__ __launch_bounds__(256) void k_fine_operator(Grid g, const double* __restrict__ kappa,
                                                       const double* __restrict__ gamma0, double h,
                                                       double omega, double alpha, int bc, int sw,
                                                       double samp, cpx<double>* __restrict__ H,
                                                       cpx<double>* __restrict__ Hs) {
  const unsigned i = node_id();
  if (i >= g.N) return;
  int c[3];
  decode(i, g, c[0], c[1], c[2]);
  const int n[3] = {g.nx, g.ny, g.nz};
  const double k = kappa[i];
  double gam = gamma0 ? gamma0[i] : 0.0;
  const bool abc = (bc == BC_ABC);
  if (abc && sw > 0) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int s = min(c[d], n[d] - 1 - c[d]);
      if (s < sw) {
        const double f = (double)(sw - s) / (double)sw;
        gam += samp * omega * f * f;
      }
    }
  }
  const double ih2 = 1.0 / (h * h);
  double scale = 1.0;
  double dre = 2.0 * DIM * ih2 - omega * omega * k * k;
  double dim_ = omega * k * k * gam;  // -beta adds +i omega kappa^2 gamma
  cpx<double> off[2 * DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool lo = c[d] == 0, hi = c[d] == n[d] - 1;
    double wm = (lo ? 0.0 : -ih2), wp = (hi ? 0.0 : -ih2);
    if (abc && (lo || hi)) {
      if (lo) wp = -2.0 * ih2;
      if (hi) wm = -2.0 * ih2;
      dim_ += 2.0 * omega * k / h;
      scale *= 0.5;
    }
    off[2 * d] = cmk(wm, 0.0);
    off[2 * d + 1] = cmk(wp, 0.0);
  }
  const size_t N = (size_t)g.N;
  H[i] = cmk(scale * dre, scale * dim_);
  Hs[i] = cmk(scale * dre, scale * (dim_ + alpha * omega * omega));
#pragma unroll
  for (int e = 0; e < 2 * DIM; ++e) {
    H[(size_t)(e + 1) * N + i] = scale * off[e];
    Hs[(size_t)(e + 1) * N + i] = scale * off[e];
  }
}

// Compact 4th-order stencil, eq. (disc4thCompact) / (disc4thCompact3D): H = L - M diag(beta)
// with the mass stencil M acting on beta u (beta of the neighbour node; the stencil is
// printed for constant kappa), H_s = H + i alpha omega^2 M.  Both as 3^DIM-box arrays
// (x fastest); weights pointing outside the grid are dropped; with bc = BC_ABC the
// absorbing layer is added to gamma (no Sommerfeld rows for this stencil).

template <int DIM>
__global__ __launch_bounds__(256) void k_fine_compact4(Grid g, const double* __restrict__ kappa,
                                                       const double* __restrict__ gamma0, double h,
                                                       double omega, double alpha, int bc, int sw,
                                                       double samp, cpx<double>* __restrict__ H,
                                                       cpx<double>* __restrict__ Hs) {
  const unsigned i = node_id();
  if (i >= g.N) return;
  int c[3];
  decode(i, g, c[0], c[1], c[2]);
  const int n[3] = {g.nx, g.ny, g.nz};
  const double ih2 = 1.0 / (h * h);
  const size_t N = (size_t)g.N;
  constexpr int K = shape_K<DIM, BOX1>();
#pragma unroll
  for (int e = 0; e < K; ++e) {
    const int dx = shape_off<DIM, BOX1>(e, 0), dy = shape_off<DIM, BOX1>(e, 1),
              dz = shape_off<DIM, BOX1>(e, 2);
    const int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
    cpx<double> hv = cmk(0.0, 0.0), sv = cmk(0.0, 0.0);
    if (inside(g, x, y, z)) {
      const int l1 = (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy) + (dz < 0 ? -dz : dz);
      const double Lw = compact_L<DIM>(l1, ih2), Mw = compact_M<DIM>(l1);
      const unsigned j = (unsigned)lin(g, x, y, z);
      const double k = kappa[j];
      double gam = gamma0 ? gamma0[j] : 0.0;
      if (bc == BC_ABC && sw > 0) {
        const int cj[3] = {x, y, z};
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int s = min(cj[d], n[d] - 1 - cj[d]);
          if (s < sw) {
            const double f = (double)(sw - s) / (double)sw;
            gam += samp * omega * f * f;
          }
        }
      }
      // beta = omega^2 kappa^2 - i omega kappa^2 gamma
      const double bre = omega * omega * k * k, bim = -omega * k * k * gam;
      hv = cmk(Lw - Mw * bre, -Mw * bim);
      sv = cmk(hv.re, hv.im + alpha * omega * omega * Mw);
    }
    H[(size_t)e * N + i] = hv;
    Hs[(size_t)e * N + i] = sv;
  }
}

hipError_t fine_compact4(int dim, Grid g, const double* kappa, const double* gamma, double h,
                         double omega, double alpha, int bc, int sw, double samp, cpx<double>* H,
                         cpx<double>* Hs, hipStream_t s) {
  const unsigned nb = nblocks(g.N, 256);
  if (dim == 2)
    k_fine_compact4<2><<<nb, 256, 0, s>>>(g, kappa, gamma, h, omega, alpha, bc, sw, samp, H, Hs);
  else
    k_fine_compact4<3><<<nb, 256, 0, s>>>(g, kappa, gamma, h, omega, alpha, bc, sw, samp, H, Hs);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t fine_operator(int dim, Grid g, const double* kappa, const double* gamma, double h,
                         double omega, double alpha, int bc, int sw, double samp, cpx<double>* H,
                         cpx<double>* Hs, hipStream_t s) {
  const unsigned nb = nblocks(g.N, 256);
  if (dim == 2)
    k_fine_operator<2><<<nb, 256, 0, s>>>(g, kappa, gamma, h, omega, alpha, bc, sw, samp, H, Hs);
  else
    k_fine_operator<3><<<nb, 256, 0, s>>>(g, kappa, gamma, h, omega, alpha, bc, sw, samp, H, Hs);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// kappa must be finite and > 0, gamma finite and >= 0; flag[0] = 1 otherwise
__global__ __launch_bounds__(256) void k_check_media(long long N, const double* __restrict__ kappa,
                                                     const double* __restrict__ gamma,
                                                     int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double k = kappa[i];
  const double g = gamma ? gamma[i] : 0.0;
  const bool ok = (k > 0.0) && (k < 1e300) && (g >= 0.0) && (g < 1e300);
  if (!ok) flag[0] = 1;
}

hipError_t check_media(long long N, const double* kappa, const double* gamma, int* flag,
                       hipStream_t s) {
  k_check_media<<<nblocks(N, 256), 256, 0, s>>>(N, kappa, gamma, flag);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// (A x)_i at node i = (cx, cy, cz), accumulated in TC.  Shared by the stencil sweep and
// the kernels that form the residual on the fly, so that both give the same bits.
template <int DIM, int SHAPE, class TC, class TX>
__device__ __forceinline__ cpx<TC> stencil_acc(const Grid& g, const cpx<TC>* __restrict__ A,
                                               const cpx<TX>* x, long long i, int cx, int cy,
                                               int cz) {
  constexpr int K = shape_K<DIM, SHAPE>();
  const size_t N = (size_t)g.N;
  cpx<TC> acc = cmk<TC>(0, 0);
  if (SHAPE == CROSS && g.offrule != 0) {
    // the 5/7-point operator with fixed off-diagonals (the values the fine operator
    // stores, so the result is the same): only the centre coefficient is read
    const int c[3] = {cx, cy, cz}, n[3] = {g.nx, g.ny, g.nz};
    double scale = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (g.offrule == 2 && (c[d] == 0 || c[d] == n[d] - 1)) scale *= 0.5;
    acc = cfma(A[i], ccast<TC>(x[i]), acc);
#pragma unroll
    for (int k = 1; k < K; ++k) {
      const int d = (k - 1) / 2;
      const bool up = ((k - 1) & 1) != 0;
      const int dx = shape_off<DIM, SHAPE>(k, 0), dy = shape_off<DIM, SHAPE>(k, 1),
                dz = shape_off<DIM, SHAPE>(k, 2);
      // a neighbour outside the grid: the node's own value with weight 0 (no branch)
      const bool ok = inside(g, cx + dx, cy + dy, cz + dz);
      const bool lo = c[d] == 0, hi = c[d] == n[d] - 1;
      const double wv = (g.offrule == 2 && ((up && lo) || (!up && hi))) ? -2.0 * g.ih2 : -g.ih2;
      const TC ov = ok ? (TC)(scale * wv) : (TC)0;
      const long long j = ok ? i + dx + (long long)g.nx * (dy + (long long)g.ny * dz) : i;
      const cpx<TC> xv = ccast<TC>(x[j]);
      acc.re = fma(ov, xv.re, acc.re);
      acc.im = fma(ov, xv.im, acc.im);
    }
  } else {
    // a coefficient that points outside the grid is an exact zero, so its term is taken
    // with the node's own value in place of the missing neighbour: every load is issued
    // unconditionally and the loads of all K terms can be in flight together
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int dx = shape_off<DIM, SHAPE>(k, 0), dy = shape_off<DIM, SHAPE>(k, 1),
                dz = shape_off<DIM, SHAPE>(k, 2);
      const bool ok = inside(g, cx + dx, cy + dy, cz + dz);
      const long long j = ok ? i + dx + (long long)g.nx * (dy + (long long)g.ny * dz) : i;
      acc = cfma(A[(size_t)k * N + i], ccast<TC>(x[j]), acc);
    }
  }
  return acc;
}

// the residual at tile node (gx, gy, gz), zero outside the grid: evaluated at the node
// clamped into the grid, so that no load depends on a branch
template <int DIM, int SHAPE, class T>
__device__ __forceinline__ cpx<T> resid_tile(const Grid& g, const cpx<T>* __restrict__ A,
                                             const cpx<T>* __restrict__ q, const cpx<T>* u,
                                             bool valid, int gx, int gy, int gz) {
  const bool in = valid && inside(g, gx, gy, gz);
  const int cx = min(max(gx, 0), g.nx - 1), cy = min(max(gy, 0), g.ny - 1);
  const int cz = (DIM == 3) ? min(max(gz, 0), g.nz - 1) : 0;
  const cpx<T> rv = resid_at<DIM, SHAPE, T>(g, A, q, u, lin(g, cx, cy, cz), cx, cy, cz);
  return in ? rv : cmk<T>(0, 0);
}

// the residual q - A u at node i, in T (the value the OP_RESID sweep stores)
template <int DIM, int SHAPE, class T>
__device__ __forceinline__ cpx<T> resid_at(const Grid& g, const cpx<T>* __restrict__ A,
                                           const cpx<T>* __restrict__ q, const cpx<T>* u,
                                           long long i, int cx, int cy, int cz) {
  return q[i] - stencil_acc<DIM, SHAPE, T, T>(g, A, u, i, cx, cy, cz);
}

// ------------------------------------------------------------------ stencil sweep
// y = A x (APPLY), y = b - A x (RESID), y += A x (ADD); A stored [K][N] in TC,
// accumulation in TC.  Coefficients that point outside the grid are zero by
// construction, so those neighbours are skipped.
template <int DIM, int SHAPE, int MODE, class TC, class TX, class TY>
__global__ __launch_bounds__(256) void k_stencil(Grid g, const cpx<TC>* __restrict__ A,
                                                 const cpx<TX>* __restrict__ x,
                                                 const cpx<TY>* __restrict__ b,
                                                 cpx<TY>* __restrict__ y) {
  const unsigned i = node_id();
  if (i >= g.N) return;
  int cx, cy, cz;
  decode(i, g, cx, cy, cz);
  const cpx<TC> acc = stencil_acc<DIM, SHAPE, TC, TX>(g, A, x, (long long)i, cx, cy, cz);
  if (MODE == OP_APPLY) {
    y[i] = ccast<TY>(acc);
  } else if (MODE == OP_RESID) {
    y[i] = ccast<TY>(ccast<TC>(b[i]) - acc);
  } else {
    y[i] = ccast<TY>(ccast<TC>(y[i]) + acc);
  }
}

template <int DIM, int SHAPE, class TC, class TX, class TY>
static hipError_t stencil_t(Grid g, int mode, const void* A, const void* x, const void* b, void* y,
                            hipStream_t s) {
  const unsigned nb = nblocks(g.N, 256);
  auto Ap = (const cpx<TC>*)A;
  auto xp = (const cpx<TX>*)x;
  auto bp = (const cpx<TY>*)b;
  auto yp = (cpx<TY>*)y;
  if (mode == OP_APPLY)
    k_stencil<DIM, SHAPE, OP_APPLY, TC, TX, TY><<<nb, 256, 0, s>>>(g, Ap, xp, bp, yp);
  else if (mode == OP_RESID)
    k_stencil<DIM, SHAPE, OP_RESID, TC, TX, TY><<<nb, 256, 0, s>>>(g, Ap, xp, bp, yp);
  else
    k_stencil<DIM, SHAPE, OP_ADD, TC, TX, TY><<<nb, 256, 0, s>>>(g, Ap, xp, bp, yp);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

template <int DIM, int SHAPE>
static hipError_t stencil_p(Grid g, int mode, int pc, const void* A, int px, const void* x, int py,
                            const void* b, void* y, hipStream_t s) {
  if (pc == PREC_F64 && px == PREC_F64 && py == PREC_F64)
    return stencil_t<DIM, SHAPE, double, double, double>(g, mode, A, x, b, y, s);
  if (pc == PREC_F32 && px == PREC_F32 && py == PREC_F32)
    return stencil_t<DIM, SHAPE, float, float, float>(g, mode, A, x, b, y, s);
  if (pc == PREC_F64 && px == PREC_F32 && py == PREC_F64)
    return stencil_t<DIM, SHAPE, double, float, double>(g, mode, A, x, b, y, s);
  return hipErrorInvalidValue;
}

hipError_t stencil(int dim, int shape, Grid g, int mode, int pc, const void* A, int px,
                   const void* x, int py, const void* b, void* y, hipStream_t s) {
  if (dim == 2) {
    if (shape == CROSS) return stencil_p<2, CROSS>(g, mode, pc, A, px, x, py, b, y, s);
    if (shape == BOX1) return stencil_p<2, BOX1>(g, mode, pc, A, px, x, py, b, y, s);
    if (shape == BOX2) return stencil_p<2, BOX2>(g, mode, pc, A, px, x, py, b, y, s);
    if (shape == BOX3) return stencil_p<2, BOX3>(g, mode, pc, A, px, x, py, b, y, s);
  } else {
    if (shape == CROSS) return stencil_p<3, CROSS>(g, mode, pc, A, px, x, py, b, y, s);
    if (shape == BOX1) return stencil_p<3, BOX1>(g, mode, pc, A, px, x, py, b, y, s);
    if (shape == BOX2) return stencil_p<3, BOX2>(g, mode, pc, A, px, x, py, b, y, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ additive Vanka apply
// Sec. 3.2, eq. (smoother): u <- u + w sum_c V_c^T W_c A_c^{-1} V_c r.  Written as a
// gather at the destination node i: node i is member a of the patch anchored at
// c = i - off_a, whose local solve contributes row a of A_c^{-1} times r on the
// members c + off_m.  G[(a*Np + m)][i] = (w / cnt_i) (A_{i-off_a}^{-1})[a][m]
// (zero where the patch or the member does not exist), so
//     u_i += sum_{a,m} G[(a*Np+m)][i] * r[i - off_a + off_m].
// Every patch inverse entry is read exactly once per sweep; no atomics.
// 2D: the 5x5 neighbourhood of r is loaded once into registers.
// Streaming loads of the patch inverses: read once per sweep, so they are loaded
// non-temporally to leave L2 / MALL to the vectors.
template <class T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load((const v2*)p);
  return cmk<T>(v.x, v.y);
}

// Tile of the sweep: TX x TY nodes (x, y) in one z-plane; each wavefront covers 64
// consecutive nodes of one grid row, so every load of the smoother entries is one
// contiguous 64-node run.  The residual is staged in LDS with a halo of 2 (patch
// radius 1 + member radius 1).
constexpr int VT_X = 64, VT_Y = 4, VT_H = 2;

// Smoother entry sets: the per-patch form (entry a*Np + m reads r at off_m - off_a)
// and the assembled form (the 5^DIM box).
enum SmForm : int { SM_FULL = 0, SM_POINT = 1, SM_BOX2 = 2, SM_PLUS = 3, SM_RB = 4, SM_ELEMENT = 5 };

template <int DIM, int FORM>
__host__ __device__ constexpr int sm_entries() {
  return FORM == SM_BOX2 ? shape_K<DIM, BOX2>() : patch_Np<DIM, FORM>() * patch_Np<DIM, FORM>();
}
template <int DIM, int FORM>
__host__ __device__ constexpr int sm_off(int e, int c) {
  return FORM == SM_BOX2 ? shape_off<DIM, BOX2>(e, c)
                         : patch_off<DIM, FORM>(e % patch_Np<DIM, FORM>(), c) -
                               patch_off<DIM, FORM>(e / patch_Np<DIM, FORM>(), c);
}

// RS >= 0 (the stencil shape of A): the residual is formed in the tile stage from
// r := q, A and u_in (q - A u_in at every tile node, halo included), and the result
// u_in + B (q - A u_in) goes to u, a different array (the halo reads u_in of the
// neighbouring tiles, so the update cannot be in place).  RS < 0: r is read, and u is
// updated in place (u_in unused).
template <int DIM, int FORM, bool ZERO, class T, int RS = -1>
__global__ __launch_bounds__(256) void k_vanka_sweep(Grid g, const cpx<T>* __restrict__ G,
                                                     const cpx<T>* __restrict__ r,
                                                     cpx<T>* __restrict__ u,
                                                     const cpx<T>* __restrict__ A = nullptr,
                                                     const cpx<T>* u_in = nullptr) {
  constexpr int SX = VT_X + 2 * VT_H, SY = VT_Y + 2 * VT_H, SZ = (DIM == 3) ? 1 + 2 * VT_H : 1;
  constexpr int HZ = (DIM == 3) ? VT_H : 0;
  __shared__ cpx<T> tile[SZ * SY * SX];
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (g.nx + VT_X - 1) / VT_X, nby = (g.ny + VT_Y - 1) / VT_Y;
  const int bx = (int)(b % (unsigned)nbx), by = (int)((b / (unsigned)nbx) % (unsigned)nby);
  const int bz = (int)(b / (unsigned)(nbx * nby));
  const int x0 = bx * VT_X, y0 = by * VT_Y, z0 = bz;
  // all loads of the residual tile are issued before the first LDS write; the barrier
  // orders LDS only, so the smoother-entry loads below may start before it
  constexpr int NTL = SX * SY * SZ, NPT = (NTL + VT_X * VT_Y - 1) / (VT_X * VT_Y);
  if constexpr (RS >= 0) {
    // one residual per lane at a time (its 2K + 1 loads in flight together), written
    // straight to the tile
#pragma unroll 1
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * VT_Y * k;
      const int tx = e % SX, ty = (e / SX) % SY, tz = e / (SX * SY);
      const int gx = x0 + tx - VT_H, gy = y0 + ty - VT_H, gz = z0 + tz - HZ;
      const cpx<T> v = resid_tile<DIM, RS, T>(g, A, r, u_in, e < NTL, gx, gy, gz);
      if (e < NTL) tile[e] = v;
    }
  } else {
    cpx<T> tv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * VT_Y * k;
      const int tx = e % SX, ty = (e / SX) % SY, tz = e / (SX * SY);
      const int gx = x0 + tx - VT_H, gy = y0 + ty - VT_H, gz = z0 + tz - HZ;
      tv[k] = (e < NTL && inside(g, gx, gy, gz)) ? r[lin(g, gx, gy, gz)] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * VT_Y * k;
      if (e < NTL) tile[e] = tv[k];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const int lx = threadIdx.x % VT_X, ly = threadIdx.x / VT_X;
  const int x = x0 + lx, y = y0 + ly, z = z0;
  if (x >= g.nx || y >= g.ny) return;
  const long long i = lin(g, x, y, z);
  const long long ip = linp(g, x, y, z);
  constexpr int E = sm_entries<DIM, FORM>();
  // 3D per-patch form: three patches (81 entries) per iteration, to bound register use;
  // there plain loads keep more of them in flight than non-temporal ones
  constexpr int UNR = (DIM == 3 && FORM == SM_FULL) ? 81
                      : (E > 128 ? patch_Np<DIM, FORM>() : E);
  constexpr bool NT = (UNR == E);
  const size_t Np = (size_t)g.Np;
  const cpx<T>* t0 = tile + (HZ * SY + (ly + VT_H)) * SX + (lx + VT_H);
  cpx<T> acc = cmk<T>(0, 0);
  if constexpr (DIM == 2 && FORM == SM_FULL && sizeof(T) == 8 && RS < 0) {
    // 81 complex128 entries: in one sequence the compiler issues the loads one at a time,
    // each waited for; in groups of 16, issued together before the group's products, a
    // group is in flight at once (same summation order)
    constexpr int NG = 16;
    static_for<0, (E + NG - 1) / NG>([&](auto gc) {
      constexpr int e0 = decltype(gc)::value * NG, ne = (E - e0) < NG ? (E - e0) : NG;
      cpx<T> gv[ne];
      static_for<0, ne>([&](auto kc) {
        gv[decltype(kc)::value] = ld_stream(G + (size_t)(e0 + decltype(kc)::value) * Np + ip);
      });
      // pins the group's loads ahead of its products (the scheduler would otherwise move
      // each load down to its product)
#pragma unroll
      for (int k = 0; k < ne; ++k) asm volatile("" : "+v"(gv[k].re), "+v"(gv[k].im));
      static_for<0, ne>([&](auto kc) {
        constexpr int e = e0 + decltype(kc)::value;
        constexpr int dx = sm_off<DIM, FORM>(e, 0), dy = sm_off<DIM, FORM>(e, 1);
        acc = cfma(gv[decltype(kc)::value], t0[dy * SX + dx], acc);
      });
    });
  } else {
#pragma unroll 1
    for (int e0 = 0; e0 < E; e0 += UNR) {
#pragma unroll
      for (int q = 0; q < UNR; ++q) {
        const int e = e0 + q;
        const int dx = sm_off<DIM, FORM>(e, 0), dy = sm_off<DIM, FORM>(e, 1),
                  dz = sm_off<DIM, FORM>(e, 2);
        const cpx<T> gv = NT ? ld_stream(G + (size_t)e * Np + ip) : G[(size_t)e * Np + ip];
        acc = cfma(gv, t0[(dz * SY + dy) * SX + dx], acc);
      }
    }
  }
  if constexpr (RS >= 0)
    u[i] = u_in[i] + acc;
  else
    u[i] = ZERO ? acc : (u[i] + acc);
}

// The 1x1 patch (damped point Jacobi) needs no neighbour: u_i (+)= G_i r_i, streamed
// without a residual tile.
template <bool ZERO, class T, int DIM = 2, int RS = -1>
__global__ __launch_bounds__(256) void k_point_sweep(Grid g, const cpx<T>* __restrict__ G,
                                                     const cpx<T>* __restrict__ r,
                                                     cpx<T>* __restrict__ u,
                                                     const cpx<T>* __restrict__ A = nullptr,
                                                     const cpx<T>* u_in = nullptr) {
  const unsigned i = node_id();
  if (i >= g.N) return;
  int x, y, z;
  decode(i, g, x, y, z);
  const cpx<T> d = ld_stream(G + linp(g, x, y, z));
  if constexpr (RS >= 0) {
    const cpx<T> rv = resid_at<DIM, RS, T>(g, A, r, u_in, (long long)i, x, y, z);
    u[i] = u_in[i] + cfma(d, rv, cmk<T>(0, 0));
  } else {
    const cpx<T> acc = cfma(d, r[i], cmk<T>(0, 0));
    u[i] = ZERO ? acc : (u[i] + acc);
  }
}

template <int DIM, int FORM, class T>
static hipError_t vanka_sweep_t(Grid g, const void* G, const void* r, void* u, bool zero,
                                hipStream_t s) {
  if constexpr (FORM == SM_POINT) {
    const unsigned nb = nblocks((size_t)g.N, 256);
    if (zero)
      k_point_sweep<true, T><<<nb, 256, 0, s>>>(g, (const cpx<T>*)G, (const cpx<T>*)r, (cpx<T>*)u);
    else
      k_point_sweep<false, T><<<nb, 256, 0, s>>>(g, (const cpx<T>*)G, (const cpx<T>*)r, (cpx<T>*)u);
    VH_LAUNCH_CHECK();
    return hipSuccess;
  }
  const unsigned nb = (unsigned)(((g.nx + VT_X - 1) / VT_X) * ((g.ny + VT_Y - 1) / VT_Y) * g.nz);
  if (zero)
    k_vanka_sweep<DIM, FORM, true, T><<<nb, VT_X * VT_Y, 0, s>>>(g, (const cpx<T>*)G,
                                                                 (const cpx<T>*)r, (cpx<T>*)u);
  else
    k_vanka_sweep<DIM, FORM, false, T><<<nb, VT_X * VT_Y, 0, s>>>(g, (const cpx<T>*)G,
                                                                  (const cpx<T>*)r, (cpx<T>*)u);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t vanka_sweep(int dim, int form, Grid g, int prec, const void* G, const void* r, void* u,
                       bool zero, hipStream_t s) {
#define VH_VP(D, F)                                                              \
  if (dim == D && form == F)                                                     \
    return prec == PREC_F64 ? vanka_sweep_t<D, F, double>(g, G, r, u, zero, s) \
                            : vanka_sweep_t<D, F, float>(g, G, r, u, zero, s);
  VH_VP(2, SM_FULL)
  VH_VP(3, SM_FULL)
  VH_VP(2, SM_POINT)
  VH_VP(3, SM_POINT)
  VH_VP(2, SM_BOX2)
  VH_VP(3, SM_BOX2)
  VH_VP(2, SM_PLUS)
  VH_VP(3, SM_PLUS)
  VH_VP(2, SM_RB)
  VH_VP(3, SM_RB)
  VH_VP(2, SM_ELEMENT)
  VH_VP(3, SM_ELEMENT)
#undef VH_VP
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ Vanka setup
// Sec. 3.2/3.3: for every patch c (anchored at every node, truncated at the
// boundary), A_c = V_c H_s V_c^T is inverted in FP64 by Gauss-Jordan elimination
// with partial pivoting.  One lane per patch row (Np lanes per patch; a patch of more
// than 16 members takes 32 lanes, so that it fills half a wave and its pivot search
// stays inside DPP rows); out-of-domain members are identity rows (padding).
// Pivoting is implicit: rows stay in their lanes, the pivot row of each step is
// broadcast through LDS.  Pivot rows are not normalised during the elimination: after
// step s, A^{-1}[step(L)][piv[s]] = a_L[s] / d_L for lane L, d_L the pivot value of
// row L at its step.  Row i of A_c^{-1} is written, scaled by w / cnt(c + off_i), to
// G[(i*Np + m)][c + off_i].
__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, 64); }

// f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>): a loop whose
// index is a compile-time constant in every iteration
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// is (x, y, z) the anchor of a patch?  Every node is, except for ELEMENT patches, which
// are anchored at the lowest corner of every cell
template <int DIM, int PATCH>
__device__ __forceinline__ bool anchor_ok(const Grid& g, int x, int y, int z) {
  if (PATCH != PATCH_ELEMENT) return inside(g, x, y, z);
  return (unsigned)x < (unsigned)(g.nx - 1) && (unsigned)y < (unsigned)(g.ny - 1) &&
         (DIM == 2 || (unsigned)z < (unsigned)(g.nz - 1));
}

// number of patches containing node (x, y, z) (Sec. 3.3 weights)
template <int DIM, int PATCH>
__device__ __forceinline__ int patch_count(const Grid& g, int x, int y, int z) {
  if (PATCH == PATCH_POINT) return 1;
  if (PATCH == PATCH_FULL) {
    int c = (3 - (x == 0) - (x == g.nx - 1)) * (3 - (y == 0) - (y == g.ny - 1));
    if (DIM == 3) c *= (3 - (z == 0) - (z == g.nz - 1));
    return c;
  }
  int c = 0;
#pragma unroll
  for (int k = 0; k < patch_Np<DIM, PATCH>(); ++k)
    c += anchor_ok<DIM, PATCH>(g, x - patch_off<DIM, PATCH>(k, 0), y - patch_off<DIM, PATCH>(k, 1),
                               z - patch_off<DIM, PATCH>(k, 2))
             ? 1
             : 0;
  return c;
}

// lanes per patch in the setup kernel
template <int DIM, int PATCH>
__host__ __device__ constexpr int setup_group() {
  return patch_Np<DIM, PATCH>() > 16 ? 32 : patch_Np<DIM, PATCH>();
}

// waves per block of the setup kernel: the LDS staging area (Np*Np rows of PB
// patches) must fit in 64 KB
template <int DIM, int PATCH, class T>
__host__ __device__ constexpr int setup_waves() {
  return (patch_Np<DIM, PATCH>() * patch_Np<DIM, PATCH>() * 4 * (64 / setup_group<DIM, PATCH>()) *
              (int)sizeof(cpx<T>) <= 65536)
             ? 4
             : 2;
}

// max(v, v of a partner lane) with the partner chosen by a DPP pattern: 0 = lane ^ 1,
// 1 = lane ^ 2 (quad permutes), 2 = mirror within 8 lanes, 3 = mirror within 16 lanes.
// Applied in that order, every lane ends with the maximum over its 16-lane row.
__device__ __forceinline__ unsigned dpp_max(unsigned v, int ctrl_sel) {
  unsigned o;
  switch (ctrl_sel) {
    case 0: o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false); break;
    case 1: o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false); break;
    case 2: o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false); break;
    default: o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false); break;
  }
  return o > v ? o : v;
}

// acc += c p with the FMAs of the elimination update in its order (re: c.re p.re, then
// -c.im p.im; im: c.re p.im, then c.im p.re), p = lane L of each 16-lane row of the
// register pair, read through the FMA's own row-broadcast operand.  The s_nop covers the
// wait a broadcast operand needs after a vector ALU write to it.
template <int L>
__device__ __forceinline__ void cupd_rowb(cpx<double>& acc, const cpx<double>& c,
                                          const cpx<double>& p) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %2, %4 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %3, %4 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %2, %5 row_newbcast:%6 row_mask:0xf bank_mask:0xf"
      : "+v"(acc.re), "+v"(acc.im)
      : "v"(p.re), "v"(p.im), "v"(c.re), "v"(c.im), "i"(L));
}
// the same for two entries (one wait for both)
template <int L0, int L1>
__device__ __forceinline__ void cupd2_rowb(cpx<double>& a0, cpx<double>& a1, const cpx<double>& c,
                                           const cpx<double>& p0, const cpx<double>& p1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, -%5, %9 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %4, %9 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %6, %8 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, -%7, %9 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %7, %8 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %6, %9 row_newbcast:%11 row_mask:0xf bank_mask:0xf"
      : "+v"(a0.re), "+v"(a0.im), "+v"(a1.re), "+v"(a1.im)
      : "v"(p0.re), "v"(p0.im), "v"(p1.re), "v"(p1.im), "v"(c.re), "v"(c.im), "i"(L0), "i"(L1));
}

template <int DIM, int SHAPE, int PATCH, class T, bool NOPIV = false>
__global__ __launch_bounds__(256, 1) void k_vanka_setup(Grid g, const cpx<double>* __restrict__ A,
                                                     double w, cpx<T>* __restrict__ G, Slab sl) {
  constexpr int Np = patch_Np<DIM, PATCH>();
  constexpr int GW = setup_group<DIM, PATCH>();
  constexpr int PPW = 64 / GW;
  constexpr int WPB = setup_waves<DIM, PATCH, T>();
  constexpr int PB = WPB * PPW;  // patches per block
  __shared__ cpx<T> stage[Np * Np * PB];
  __shared__ unsigned char okrow[Np * PB];
  __shared__ long long cpad[PB];  // padded index of each patch anchor
  const unsigned lane = threadIdx.x & 63u;
  const unsigned wib = threadIdx.x >> 6;  // wave in block
  const unsigned slot = lane / GW;
  const int k = (int)(lane % GW);
  const long long c0 = sl.c_lo + (long long)blockIdx.x * PB;
  const int pslot = (int)(wib * PPW + slot);
  const long long c = c0 + pslot;
  const bool in_slot = slot < (unsigned)PPW && k < Np;
  const bool in_range = in_slot && c < sl.c_hi;
  const int base = (int)(slot < (unsigned)PPW ? slot : 0) * GW;
  const size_t N = (size_t)g.N;
  int cx = 0, cy = 0, cz = 0;
  if (in_range) decode((unsigned)c, g, cx, cy, cz);
  // a node that anchors no patch keeps identity rows and writes nothing
  const bool active = in_range && anchor_ok<DIM, PATCH>(g, cx, cy, cz);
  const int kk = k < Np ? k : 0;
  const int kx = cx + patch_off<DIM, PATCH>(kk, 0), ky = cy + patch_off<DIM, PATCH>(kk, 1),
            kz = cz + patch_off<DIM, PATCH>(kk, 2);
  const bool mem_in = active && inside(g, kx, ky, kz);
  const long long ik = mem_in ? lin(g, kx, ky, kz) : 0;

  cpx<double> a[Np];
#pragma unroll
  for (int m = 0; m < Np; ++m) {
    a[m] = cmk(0.0, 0.0);
    if (mem_in) {
      const int dx = patch_off<DIM, PATCH>(m, 0) - patch_off<DIM, PATCH>(kk, 0);
      const int dy = patch_off<DIM, PATCH>(m, 1) - patch_off<DIM, PATCH>(kk, 1);
      const int dz = patch_off<DIM, PATCH>(m, 2) - patch_off<DIM, PATCH>(kk, 2);
      const int s = shape_index<DIM, SHAPE>(dx, dy, dz);
      if (s >= 0 && inside(g, kx + dx, ky + dy, kz + dz)) a[m] = A[(size_t)s * N + ik];
    } else if (m == k) {
      a[m] = cmk(1.0, 0.0);
    }
  }

  // Gauss-Jordan steps with a rotating row: at step s, a[0] holds column s of the
  // working matrix, a[1 .. Np-1-s] the columns after it and a[Np-s ..] the inverse's
  // columns of steps 0 .. s-1; every step shifts the row down by one and appends the
  // new inverse column, so the loop stays rolled and every register index is static.
  // The pivot is the unused row with the largest |re| + |im| in a[0], compared in
  // single precision with the lane index in the low mantissa bits (the first row on
  // ties within 2^-18), so that one 32-bit maximum over the patch's lanes finds it.
  // Its raw row is broadcast through LDS and every row takes
  // a[m] <- a[m+1] + c * p[m+1], a[Np-1] <- c with c = -a[0]/p[0], except the pivot
  // row: c = 0 and a[Np-1] <- 1, so it stays unnormalised and its pivot value d is
  // kept to scale the row once at the end.  The pivot sequence of each patch is kept
  // in LDS.
  // NOPIV (the patch matrix complex symmetric with a positive definite imaginary part,
  // where elimination in the natural order needs no pivoting): step s takes row s, and
  // the working matrix stays symmetric up to the scaling of the rows already used, so
  // the pivot row is assembled from every row's own leading entry: position
  // (k - s) mod Np of the pivot row is a_k[0] for a row k not yet used and -a_k[0] / d_k
  // for a used row k with pivot value d_k.  Every lane writes one entry, in one LDS
  // store, instead of the pivot lane writing all Np.
  __shared__ unsigned char pivs[PB * Np];
  __shared__ cpx<double> prow[WPB][PPW][Np];
  bool used = false;
  int mystep = k;
  cpx<double> dpiv = cmk(1.0, 0.0);
  cpx<double> ndinv = cmk(0.0, 0.0);  // -1 / d of this lane's row once used (NOPIV)
  cpx<double>* pr = prow[wib][slot < (unsigned)PPW ? slot : 0];
  constexpr int CH = 6;  // pivot-row entries read per batch
  // unrolled three steps at a time, the rotating row costs register moves at the loop edge
  // (a rotation by three); the no-pivot 3D form is unrolled whole instead
  constexpr int UNROLL = (NOPIV && GW == 32) ? Np : 3;
#pragma unroll UNROLL
  for (int s = 0; s < Np; ++s) {
    const cpx<double> as = a[0];
    int best = s;
    if constexpr (NOPIV) {
      if (in_slot) {
        const int pos = k >= s ? k - s : k - s + Np;
        pr[pos] = used ? as * ndinv : as;
      }
    } else {
    const float mag = (float)(fabs(as.re) + fabs(as.im));
    unsigned key = (in_slot && !used) ? ((__float_as_uint(mag) & ~31u) | (31u - (unsigned)k)) : 0u;
    if constexpr (GW == 32) {
      key = dpp_max(key, 0);
      key = dpp_max(key, 1);
      key = dpp_max(key, 2);
      key = dpp_max(key, 3);
      const unsigned o = (unsigned)__shfl_xor((int)key, 16, 64);
      key = o > key ? o : key;
    } else {
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) {
        if (off >= GW) continue;
        const unsigned o = (unsigned)__shfl((int)key, (int)lane + off, 64);
        key = (k + off < Np && o > key) ? o : key;
      }
      key = (unsigned)__shfl((int)key, base, 64);
    }
    best = 31 - (int)(key & 31u);
    if (in_slot && k == 0) pivs[pslot * Np + s] = (unsigned char)best;
    }
    const bool am = in_slot && (k == best);
    if (!NOPIV && am) {
#pragma unroll
      for (int m = 0; m < Np; ++m) pr[m] = a[m];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const cpx<double> ps = pr[0];
    const double dd = 1.0 / (ps.re * ps.re + ps.im * ps.im);
    const cpx<double> inv = cmk(ps.re * dd, -ps.im * dd);
    const cpx<double> c = am ? cmk(0.0, 0.0) : cmk(0.0, 0.0) - as * inv;
    if constexpr (GW % 16 == 0) {
      // a patch fills whole 16-lane rows: every row reads the pivot row once (lane
      // 16r + i entries i and 16 + i, two LDS reads per lane instead of Np - 1) and each
      // FMA takes its entry from lane m % 16 of its row through the operand broadcast
      const int li = (int)(lane & 15u);
      const cpx<double> pA = pr[li];
      const cpx<double> pB = pr[16 + li < Np ? 16 + li : 0];
      static_for<1, Np>([&](auto mi) {
        constexpr int m = decltype(mi)::value;
        if constexpr (m % 2 == 1) {
          cpx<double> t0 = a[m];
          if constexpr (m + 1 < Np) {
            cpx<double> t1 = a[m + 1];
            cupd2_rowb<m % 16, (m + 1) % 16>(t0, t1, c, m < 16 ? pA : pB, m + 1 < 16 ? pA : pB);
            a[m] = t1;
          } else {
            cupd_rowb<m % 16>(t0, c, m < 16 ? pA : pB);
          }
          a[m - 1] = t0;
        }
      });
    } else {
#pragma unroll
      for (int m0 = 0; m0 + 1 < Np; m0 += CH) {
        cpx<double> pb[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (m0 + q + 1 < Np) pb[q] = pr[m0 + q + 1];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          if (m0 + q + 1 < Np) {
            cpx<double> t;
            t.re = fma(-c.im, pb[q].im, fma(c.re, pb[q].re, a[m0 + q + 1].re));
            t.im = fma(c.im, pb[q].re, fma(c.re, pb[q].im, a[m0 + q + 1].im));
            a[m0 + q] = t;
          }
        }
      }
    }
    a[Np - 1] = am ? cmk(1.0, 0.0) : c;
    if (am) {
      used = true;
      mystep = s;
      dpiv = ps;
      ndinv = cmk(0.0, 0.0) - inv;
    }
    // every lane has read the row before the next step's pivot lane overwrites it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }
  __syncthreads();

  // this lane holds row i = mystep of the inverse; its destination is member i of c.
  // Stage the weighted row in LDS as [i*Np + m][patch], then write each of the Np*Np
  // rows for the block's PB consecutive patches as one contiguous run.
  const int i = mystep;
  int ox = 0, oy = 0, oz = 0;
#pragma unroll
  for (int q = 0; q < Np; ++q)
    if (q == i) {
      ox = patch_off<DIM, PATCH>(q, 0);
      oy = patch_off<DIM, PATCH>(q, 1);
      oz = patch_off<DIM, PATCH>(q, 2);
    }
  const int jx = cx + ox, jy = cy + oy, jz = cz + oz;
  // destination outside the grid: an out-of-domain member (or, only with
  // non-finite patch entries, an inconsistent pivot sequence)
  const bool ok = mem_in && inside(g, jx, jy, jz);
  if (in_slot) {
    const double wt = ok ? w / (double)patch_count<DIM, PATCH>(g, jx, jy, jz) : 0.0;
    const double dd = 1.0 / (dpiv.re * dpiv.re + dpiv.im * dpiv.im);
    const cpx<double> sc = cmk(wt * dpiv.re * dd, -wt * dpiv.im * dd);  // w / (cnt d)
#pragma unroll
    for (int s = 0; s < Np; ++s)
      stage[((NOPIV ? s : (int)pivs[pslot * Np + s]) + i * Np) * PB + pslot] = ccast<T>(sc * a[s]);
    okrow[i * PB + pslot] = ok ? 1 : 0;
    if (k == 0) cpad[pslot] = active ? linp(g, cx, cy, cz) : 0;
  }
  // padded-layout offset of every member, computed once per block (member k by lane k
  // of wave 0) instead of once per stored entry
  __shared__ long long moff[Np];
  if (threadIdx.x < (unsigned)Np) moff[k] = linp(g, patch_off<DIM, PATCH>(kk, 0),
                                                 patch_off<DIM, PATCH>(kk, 1),
                                                 patch_off<DIM, PATCH>(kk, 2));
  __syncthreads();
  for (int e = threadIdx.x; e < Np * Np * PB; e += blockDim.x) {
    const int r = e / PB, p = e % PB, ii = r / Np;
    if (!okrow[ii * PB + p]) continue;
    G[(size_t)r * sl.gstride + (size_t)(cpad[p] + moff[ii] - sl.gbase)] = stage[e];
  }
}

template <int DIM, int SHAPE, int PATCH, class T, bool NOPIV>
static void vanka_setup_l(Grid g, const cpx<double>* A, double w, void* G, Slab sl,
                          hipStream_t s) {
  constexpr int PPW = 64 / setup_group<DIM, PATCH>();
  constexpr int WPB = setup_waves<DIM, PATCH, T>();
  const long long nc = sl.c_hi - sl.c_lo;
  const unsigned nb = (unsigned)((nc + WPB * PPW - 1) / (WPB * PPW));
  k_vanka_setup<DIM, SHAPE, PATCH, T, NOPIV><<<nb, 64 * WPB, 0, s>>>(g, A, w, (cpx<T>*)G, sl);
}

template <int DIM, int SHAPE, int PATCH>
static hipError_t vanka_setup_s(Grid g, const cpx<double>* A, double w, int prec, void* G,
                                Slab sl, bool nopiv, hipStream_t s) {
  if (sl.c_lo < 0 || sl.c_hi > (long long)g.N || sl.c_lo >= sl.c_hi) return hipErrorInvalidValue;
  // elimination without pivoting is built for the Full patch only
  constexpr bool NP = PATCH == PATCH_FULL;
  if (prec == PREC_F64) {
    if (NP && nopiv)
      vanka_setup_l<DIM, SHAPE, PATCH, double, NP>(g, A, w, G, sl, s);
    else
      vanka_setup_l<DIM, SHAPE, PATCH, double, false>(g, A, w, G, sl, s);
  } else {
    if (NP && nopiv)
      vanka_setup_l<DIM, SHAPE, PATCH, float, NP>(g, A, w, G, sl, s);
    else
      vanka_setup_l<DIM, SHAPE, PATCH, float, false>(g, A, w, G, sl, s);
  }
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t vanka_setup(int dim, int shape, int patch, Grid g, const cpx<double>* A, double w,
                       int prec, void* G, Slab sl, hipStream_t s, bool nopiv) {
#define VH_VS(D, S, P)                            \
  if (dim == D && shape == S && patch == P) \
    return vanka_setup_s<D, S, P>(g, A, w, prec, G, sl, nopiv, s);
  VH_VS(2, CROSS, PATCH_FULL)
  VH_VS(2, BOX1, PATCH_FULL)
  VH_VS(2, BOX2, PATCH_FULL)
  VH_VS(3, CROSS, PATCH_FULL)
  VH_VS(3, BOX1, PATCH_FULL)
  VH_VS(3, BOX2, PATCH_FULL)
  VH_VS(2, CROSS, PATCH_POINT)
  VH_VS(2, BOX1, PATCH_POINT)
  VH_VS(2, BOX2, PATCH_POINT)
  VH_VS(3, CROSS, PATCH_POINT)
  VH_VS(3, BOX1, PATCH_POINT)
  VH_VS(3, BOX2, PATCH_POINT)
  VH_VS(2, BOX3, PATCH_FULL)
  VH_VS(2, BOX3, PATCH_POINT)
  VH_VS(2, BOX3, PATCH_PLUS)
  VH_VS(2, BOX3, PATCH_RB)
  VH_VS(2, BOX3, PATCH_ELEMENT)
  VH_VS(2, CROSS, PATCH_PLUS)
  VH_VS(2, BOX1, PATCH_PLUS)
  VH_VS(2, BOX2, PATCH_PLUS)
  VH_VS(3, CROSS, PATCH_PLUS)
  VH_VS(3, BOX1, PATCH_PLUS)
  VH_VS(2, CROSS, PATCH_RB)
  VH_VS(2, BOX1, PATCH_RB)
  VH_VS(2, BOX2, PATCH_RB)
  VH_VS(3, CROSS, PATCH_RB)
  VH_VS(3, BOX1, PATCH_RB)
  VH_VS(2, CROSS, PATCH_ELEMENT)
  VH_VS(2, BOX1, PATCH_ELEMENT)
  VH_VS(2, BOX2, PATCH_ELEMENT)
  VH_VS(3, CROSS, PATCH_ELEMENT)
  VH_VS(3, BOX1, PATCH_ELEMENT)
#undef VH_VS
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ symmetric assembled apply
// When H_s is complex symmetric (the 5/7-point operator, whose absorbing rows are scaled
// to keep it symmetric, and Galerkin levels built with R = c P^T), every patch matrix
// A_c = V_c H_s V_c^T and its inverse are symmetric, so the assembled smoother is
// B = D S with D = diag(w / cnt_i) and S = sum_c V_c^T A_c^{-1} V_c symmetric (Sec. 3.2,
// 3.3).  S is stored for the upper half of the 5^DIM box only: entry e' = e - C for the
// box entries e >= C (C the centre; e grows with dz, then dy, then dx, so these are the
// offsets d >= 0 in that order), S[e'][i] = S(i, i + d_e).  The sweep is then
//   u_i += D_i ( sum_{e >= C} S[e-C][i] r[i+d_e] + sum_{e > C} S[e-C][i-d_e] r[i-d_e] ),
// the second sum reading the entries stored at the neighbours i - d_e.  Blocks run x
// tiles fastest, then planes, then tile rows.  In 2D the mirrored entries lie in the same
// or the previous tile row, read a few blocks earlier, and come from L2, so each stored
// entry leaves HBM about once.  In 3D those at planes z-1 and z-2 were read by blocks a few
// dispatches earlier, but with every XCD streaming many blocks its L2 has turned over by
// then: the second read comes back from the fabric and the 3D sweep is slower than the
// full stencil (measured; keeping that reuse needs the products held on chip).

template <int DIM>
__host__ __device__ constexpr int sym_entries() { return (ipow(5, DIM) + 1) / 2; }

// rows per tile of the symmetric sweep (the residual tile stays within 33 KB / 65 KB)
template <class T>
__host__ __device__ constexpr int sym_ty() { return sizeof(T) == 4 ? 8 : 4; }

constexpr int SYM_GROUP = 16;

template <int DIM, bool ZERO, class T, int RS = -1>
__global__ __launch_bounds__(512) void k_vanka_sweep_sym(Grid g, const cpx<T>* __restrict__ S,
                                                         double w, const cpx<T>* __restrict__ r,
                                                         cpx<T>* __restrict__ u,
                                                         const cpx<T>* __restrict__ A = nullptr,
                                                         const cpx<T>* u_in = nullptr) {
  constexpr int TY = sym_ty<T>();
  constexpr int SX = VT_X + 2 * VT_H, SY = TY + 2 * VT_H, SZ = (DIM == 3) ? 1 + 2 * VT_H : 1;
  constexpr int HZ = (DIM == 3) ? VT_H : 0;
  __shared__ cpx<T> tile[SZ * SY * SX];
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (g.nx + VT_X - 1) / VT_X;
  // x tile fastest, then the plane, then the tile row
  const int bx = (int)(b % (unsigned)nbx);
  const unsigned t = b / (unsigned)nbx;
  const int bz = (int)(t % (unsigned)g.nz), by = (int)(t / (unsigned)g.nz);
  const int x0 = bx * VT_X, y0 = by * TY, z0 = bz;
  constexpr int NTL = SX * SY * SZ, NPT = (NTL + VT_X * TY - 1) / (VT_X * TY);
  if constexpr (RS >= 0) {
    // one residual per lane at a time (its 2K + 1 loads in flight together), written
    // straight to the tile
#pragma unroll 1
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * TY * k;
      const int tx = e % SX, ty = (e / SX) % SY, tz = e / (SX * SY);
      const int gx = x0 + tx - VT_H, gy = y0 + ty - VT_H, gz = z0 + tz - HZ;
      const cpx<T> v = resid_tile<DIM, RS, T>(g, A, r, u_in, e < NTL, gx, gy, gz);
      if (e < NTL) tile[e] = v;
    }
  } else {
    cpx<T> tv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * TY * k;
      const int tx = e % SX, ty = (e / SX) % SY, tz = e / (SX * SY);
      const int gx = x0 + tx - VT_H, gy = y0 + ty - VT_H, gz = z0 + tz - HZ;
      tv[k] = (e < NTL && inside(g, gx, gy, gz)) ? r[lin(g, gx, gy, gz)] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = (int)threadIdx.x + VT_X * TY * k;
      if (e < NTL) tile[e] = tv[k];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const int lx = threadIdx.x % VT_X, ly = threadIdx.x / VT_X;
  const int x = x0 + lx, y = y0 + ly, z = z0;
  if (x >= g.nx || y >= g.ny) return;
  const long long i = lin(g, x, y, z);
  const long long ip = linp(g, x, y, z);
  constexpr int K5 = ipow(5, DIM), C = (K5 - 1) / 2, EH = sym_entries<DIM>();
  const size_t Np = (size_t)g.Np;
  const int sy = g.nxp, sz = g.nxp * g.ny;
  const unsigned ipu = (unsigned)ip;  // padded index < 2^31 (checked on the host)
  const cpx<T>* t0 = tile + (HZ * SY + (ly + VT_H)) * SX + (lx + VT_H);
  cpx<T> acc = cmk<T>(0, 0);
  // own entries: S(i, i + d), d >= 0; the plane base is uniform, the per-lane part a
  // 32-bit offset.  Mirrored entries: S(i - d, i) stored at i - d, d > 0 (cached loads:
  // which of the two reads of an entry comes first depends on the tile order).  A
  // neighbour i - d outside the grid has r = 0 in the tile, so its entry only has to be
  // finite: the address stays inside the allocation (a zero guard of sym_guard() entries
  // precedes plane 0; earlier planes otherwise) and every load is unconditional.  In 3D
  // the loads go in groups of SYM_GROUP, each group issued before its products, so that
  // a group is in flight together (in one sequence the loads are otherwise issued one at
  // a time, each waited for).
  constexpr int NG = DIM == 3 ? SYM_GROUP : 2 * EH;
  static_for<0, (2 * EH - 1 + NG - 1) / NG>([&](auto gc) {
    constexpr int j0 = decltype(gc)::value * NG;
    constexpr int nj = (2 * EH - 1 - j0) < NG ? (2 * EH - 1 - j0) : NG;
    // sequence j: the own entry q = j for j < EH, then the mirrored entry q = j - EH + 1
    cpx<T> sv[nj];
    static_for<0, nj>([&](auto kc) {
      constexpr int j = j0 + decltype(kc)::value;
      constexpr int q = j < EH ? j : j - EH + 1;
      constexpr int dx = shape_off<DIM, BOX2>(C + q, 0), dy = shape_off<DIM, BOX2>(C + q, 1),
                    dz = shape_off<DIM, BOX2>(C + q, 2);
      const cpx<T>* Sq = S + (size_t)q * Np;
      sv[decltype(kc)::value] =
          j < EH ? Sq[ipu] : (Sq - (long long)(dx + sy * dy + sz * dz))[ipu];
    });
    static_for<0, nj>([&](auto kc) {
      constexpr int j = j0 + decltype(kc)::value;
      constexpr int q = j < EH ? j : j - EH + 1;
      constexpr int dx = shape_off<DIM, BOX2>(C + q, 0), dy = shape_off<DIM, BOX2>(C + q, 1),
                    dz = shape_off<DIM, BOX2>(C + q, 2);
      constexpr int to = (dz * SY + dy) * SX + dx;
      acc = cfma(sv[decltype(kc)::value], t0[j < EH ? to : -to], acc);
    });
  });
  const T dw = (T)(w / (double)patch_count<DIM, PATCH_FULL>(g, x, y, z));
  acc = cmk<T>(dw * acc.re, dw * acc.im);
  if constexpr (RS >= 0)
    u[i] = u_in[i] + acc;
  else
    u[i] = ZERO ? acc : (u[i] + acc);
}

template <int DIM, class T>
static hipError_t vanka_sweep_sym_t(Grid g, const void* S, double w, const void* r, void* u,
                                    bool zero, hipStream_t s) {
  constexpr int TY = sym_ty<T>();
  const unsigned nbx = (unsigned)((g.nx + VT_X - 1) / VT_X), nby = (unsigned)((g.ny + TY - 1) / TY);
  const unsigned nb = nbx * nby * (unsigned)g.nz;
  if (zero)
    k_vanka_sweep_sym<DIM, true, T><<<nb, VT_X * TY, 0, s>>>(g, (const cpx<T>*)S, w,
                                                             (const cpx<T>*)r, (cpx<T>*)u);
  else
    k_vanka_sweep_sym<DIM, false, T><<<nb, VT_X * TY, 0, s>>>(g, (const cpx<T>*)S, w,
                                                              (const cpx<T>*)r, (cpx<T>*)u);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// entries before plane 0 that the mirrored loads of the sweep may touch
long long sym_guard(const Grid& g) {
  return 2 + 2LL * g.nxp + (g.dim == 3 ? 2LL * g.nxp * g.ny : 0);
}

// entries after the last plane that the mirrored loads of the 3D sweep may touch
long long sym_tail(const Grid& g) { return g.dim == 3 ? 2 + 2LL * g.nxp : 0; }

// 3D form of the symmetric-half sweep, walked along z.  A block takes a 32 x 8 column of
// nodes through a chunk of zc >= 2 planes (6 by default).  At plane z each lane reads the
// 63 stored entries of its node once for its own terms, S(i, i + d) r(i + d), and, in the
// same step, the entries stored at the nodes i - d of plane z for the mirrored terms
// S(i - d, i) r(i - d) of the targets i in planes z, z + 1, z + 2: those loads touch the
// lines the neighbouring lanes of the block are loading for their own terms at that
// moment, so they come from the caches instead of reaching back two planes.  The mirrored
// sums of the next two planes ride along in registers.  Those a chunk collects for the
// first two planes of the next chunk go to `carry` (two planes per chunk boundary, x
// fastest), and sym_carry_add() adds them once every chunk is done.  The residual planes
// z .. z + 2 (with a halo of 2, zero outside the grid) sit in a four-slot LDS ring; the
// slot of plane z + 3 is filled while plane z is summed.  One stencil row (5 own and 5
// mirrored loads) per iteration keeps 62 VGPRs and 8 waves per SIMD.  At 257^3, tiles of
// 64 x 8, 64 x 4, 32 x 16 and 16 x 16 measured up to 4 % slower than this one; chunks of 6
// planes 2.5 % faster than 8, of 3 to 5 planes and 12 to 43 planes slower (4 varied by
// 8 % from one allocation of the level to the next).
constexpr int SZ_TX = 32, SZ_TY = 8;

template <bool ZERO, class T>
__global__ __launch_bounds__(SZ_TX * SZ_TY) void k_vanka_sweep_sym3z(Grid g,
                                                                    const cpx<T>* __restrict__ S,
                                                                    double w,
                                                                    const cpx<T>* __restrict__ r,
                                                                    cpx<T>* __restrict__ u,
                                                                    int zc,
                                                                    cpx<T>* __restrict__ carry) {
  constexpr int RX = SZ_TX + 4, RY = SZ_TY + 4, NR = RX * RY, NT = SZ_TX * SZ_TY;
  constexpr int NRT = (NR + NT - 1) / NT;
  __shared__ cpx<T> ring[4][NR];
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (g.nx + SZ_TX - 1) / SZ_TX, nby = (g.ny + SZ_TY - 1) / SZ_TY;
  const int bx = (int)(b % (unsigned)nbx), by = (int)((b / (unsigned)nbx) % (unsigned)nby);
  const int bz = (int)(b / (unsigned)(nbx * nby));
  const int x0 = bx * SZ_TX, y0 = by * SZ_TY;
  const int z0 = bz * zc, z1 = min(z0 + zc, g.nz);
  const int lx = (int)threadIdx.x % SZ_TX, ly = (int)threadIdx.x / SZ_TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool own = x < g.nx && y < g.ny;
  const int xc = min(x, g.nx - 1), yc = min(y, g.ny - 1);  // idle lanes load for a grid node
  const size_t Np = (size_t)g.Np;
  cpx<T> rv[NRT];
  auto fetch = [&](int zz) {
#pragma unroll
    for (int k = 0; k < NRT; ++k) {
      const int e = (int)threadIdx.x + NT * k;
      const int gx = x0 + e % RX - 2, gy = y0 + e / RX - 2;
      rv[k] = (e < NR && inside(g, gx, gy, zz)) ? r[lin(g, gx, gy, zz)] : cmk<T>(0, 0);
    }
  };
  auto store = [&](int zz) {
#pragma unroll
    for (int k = 0; k < NRT; ++k) {
      const int e = (int)threadIdx.x + NT * k;
      if (e < NR) ring[zz & 3][e] = rv[k];
    }
  };
  fetch(z0);
  store(z0);
  fetch(z0 + 1);
  store(z0 + 1);
  fetch(z0 + 2);
  store(z0 + 2);
  __syncthreads();
  cpx<T> m0 = cmk<T>(0, 0), m1 = cmk<T>(0, 0), m2 = cmk<T>(0, 0);
  const int tix = (ly + 2) * RX + (lx + 2);
  unsigned ipu = 0;  // padded index of (xc, yc, z) < 2^31 (checked on the host)
  cpx<T> acc = cmk<T>(0, 0);
  // one stencil row (dy, DZ) of the half, dx = DXLO .. 2 (entry q = 25 DZ + 5 dy + dx):
  // the node's own terms S(i, i + d) r(i + d), and the mirrored terms, where the source
  // (x - dx, y - dy) of plane z gives S(i - d, i) r(i - d) to the target of plane z + DZ.
  // A source outside the grid has r = 0 in the ring, so its entry only has to be finite:
  // the address, the lane's index shifted by a block-uniform amount, stays inside the
  // allocation (zero guards before plane 0 and after the last plane, earlier or later
  // rows and planes otherwise) and one 32-bit lane offset serves every load.
  auto row = [&](auto dzc, auto dxlo, int z, int dy) {
    constexpr int DZ = decltype(dzc)::value, DXLO = decltype(dxlo)::value;
    const cpx<T>* S0 = S + (long long)(25 * DZ + 5 * dy) * (long long)Np;
    const cpx<T>* ro = ring[(z + DZ) & 3] + tix + dy * RX;
    const cpx<T>* rm = ring[z & 3] + tix - dy * RX;
    const long long sh = (long long)g.nxp * dy;
    constexpr int NE = 3 - DXLO;
    // the row's loads first, then its products, so that they are in flight together
    cpx<T> so[NE], sm[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int dx = DXLO + k;
      const cpx<T>* Sq = S0 + (long long)dx * (long long)Np;
      so[k] = Sq[ipu];
      sm[k] = (Sq - (sh + dx))[ipu];
    }
    cpx<T>& m = DZ == 0 ? m0 : (DZ == 1 ? m1 : m2);
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int dx = DXLO + k;
      acc = cfma(so[k], ro[dx], acc);
      if (DZ > 0 || DXLO < 0 || dx > 0) m = cfma(sm[k], rm[-dx], m);
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using IM2 = std::integral_constant<int, -2>;
  for (int z = z0; z < z1; ++z) {
    fetch(z + 3);
    ipu = (unsigned)(xc + g.nxp * (yc + g.ny * z));
    acc = cmk<T>(0, 0);
    row(I0{}, I0{}, z, 0);
#pragma unroll 1
    for (int dy = 1; dy <= 2; ++dy) row(I0{}, IM2{}, z, dy);
#pragma unroll 1
    for (int dy = -2; dy <= 2; ++dy) row(I1{}, IM2{}, z, dy);
#pragma unroll 1
    for (int dy = -2; dy <= 2; ++dy) row(I2{}, IM2{}, z, dy);
    if (own) {
      const T dw = (T)(w / (double)patch_count<3, PATCH_FULL>(g, x, y, z));
      const cpx<T> t = acc + m0;
      const cpx<T> v = cmk<T>(dw * t.re, dw * t.im);
      const long long i = lin(g, x, y, z);
      u[i] = ZERO ? v : (u[i] + v);
    }
    m0 = m1;
    m1 = m2;
    m2 = cmk<T>(0, 0);
    store(z + 3);
    __syncthreads();
  }
  // m0, m1: the mirrored sums of planes z1, z1 + 1 from this chunk's planes
  if (own && z1 < g.nz) {
    const size_t plane = (size_t)g.nx * g.ny, at = (size_t)x + (size_t)g.nx * y;
    cpx<T>* c = carry + (size_t)bz * 2 * plane + at;
    c[0] = m0;
    if (z1 + 1 < g.nz) c[plane] = m1;
  }
}

// u += (w / cnt) * carry at the first two planes of every chunk but the first
template <class T>
__global__ __launch_bounds__(256) void k_sym_carry_add(Grid g, double w, int zc,
                                                       const cpx<T>* __restrict__ carry,
                                                       cpx<T>* __restrict__ u) {
  const size_t plane = (size_t)g.nx * g.ny;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = (g.nz + zc - 1) / zc;
  if (t >= (size_t)(nb - 1) * 2 * plane) return;
  const int j = (int)(t / (2 * plane)), k = (int)((t / plane) % 2);
  const int at = (int)(t % plane);
  const int x = at % g.nx, y = at / g.nx, z = (j + 1) * zc + k;
  if (z >= g.nz) return;
  const cpx<T> c = carry[t];
  const T dw = (T)(w / (double)patch_count<3, PATCH_FULL>(g, x, y, z));
  const long long i = lin(g, x, y, z);
  u[i] = u[i] + cmk<T>(dw * c.re, dw * c.im);
}

long long sym_carry_elems(const Grid& g, int planes) {
  if (g.dim != 3 || planes < 2) return 0;
  return (long long)((g.nz + planes - 1) / planes - 1) * 2 * g.nx * g.ny;
}

template <class T>
static hipError_t vanka_sweep_sym3z_t(Grid g, const void* S, double w, const void* r, void* u,
                                      bool zero, int zc, void* carry, hipStream_t s) {
  const unsigned nb = (unsigned)(((g.nx + SZ_TX - 1) / SZ_TX) * ((g.ny + SZ_TY - 1) / SZ_TY) *
                                 ((g.nz + zc - 1) / zc));
  if (zero)
    k_vanka_sweep_sym3z<true, T><<<nb, SZ_TX * SZ_TY, 0, s>>>(
        g, (const cpx<T>*)S, w, (const cpx<T>*)r, (cpx<T>*)u, zc, (cpx<T>*)carry);
  else
    k_vanka_sweep_sym3z<false, T><<<nb, SZ_TX * SZ_TY, 0, s>>>(
        g, (const cpx<T>*)S, w, (const cpx<T>*)r, (cpx<T>*)u, zc, (cpx<T>*)carry);
  VH_LAUNCH_CHECK();
  const long long nc = sym_carry_elems(g, zc);
  if (nc > 0) {
    k_sym_carry_add<T><<<nblocks(nc, 256), 256, 0, s>>>(g, w, zc, (const cpx<T>*)carry,
                                                         (cpx<T>*)u);
    VH_LAUNCH_CHECK();
  }
  return hipSuccess;
}

int sym_walk_planes(const Grid& g) {
  if (g.dim != 3) return -1;
  const long long cols = (long long)((g.nx + SZ_TX - 1) / SZ_TX) * ((g.ny + SZ_TY - 1) / SZ_TY);
  return cols * ((g.nz + SYM_WALK_PLANES - 1) / SYM_WALK_PLANES) >= SYM_WALK_MIN_BLOCKS
             ? SYM_WALK_PLANES
             : -1;
}

hipError_t vanka_sweep_sym(int dim, Grid g, int prec, const void* S, double w, const void* r,
                           void* u, bool zero, hipStream_t s, int planes, void* carry) {
  if (g.Np >= (1LL << 31)) return hipErrorInvalidValue;  // 32-bit lane offsets
  if (dim == 2)
    return prec == PREC_F64 ? vanka_sweep_sym_t<2, double>(g, S, w, r, u, zero, s)
                            : vanka_sweep_sym_t<2, float>(g, S, w, r, u, zero, s);
  if (dim != 3) return hipErrorInvalidValue;
  if (planes == 0) planes = sym_walk_planes(g);
  if (planes < 0)
    return prec == PREC_F64 ? vanka_sweep_sym_t<3, double>(g, S, w, r, u, zero, s)
                            : vanka_sweep_sym_t<3, float>(g, S, w, r, u, zero, s);
  if (planes < 2 || (sym_carry_elems(g, planes) > 0 && !carry)) return hipErrorInvalidValue;
  return prec == PREC_F64 ? vanka_sweep_sym3z_t<double>(g, S, w, r, u, zero, planes, carry, s)
                          : vanka_sweep_sym3z_t<float>(g, S, w, r, u, zero, planes, carry, s);
}

// u_out = u_in + B (q - A u_in) in one launch (2D; the residual is formed in the sweep's
// tile stage).  A 3D tile with its halo of two planes holds about ten times the nodes it
// updates, so forming the residual there would cost more stencil loads than the separate
// residual sweep saves; 3D keeps the two launches.
template <int FORM, int RS, class T>
static hipError_t fused_sweep_t(Grid g, const void* G, const void* A, const void* q,
                                const void* u_in, void* u_out, hipStream_t s) {
  auto Gp = (const cpx<T>*)G;
  auto Ap = (const cpx<T>*)A;
  auto qp = (const cpx<T>*)q;
  auto ui = (const cpx<T>*)u_in;
  auto uo = (cpx<T>*)u_out;
  if constexpr (FORM == SM_POINT) {
    k_point_sweep<false, T, 2, RS><<<nblocks((size_t)g.N, 256), 256, 0, s>>>(g, Gp, qp, uo, Ap, ui);
  } else {
    const unsigned nb = (unsigned)(((g.nx + VT_X - 1) / VT_X) * ((g.ny + VT_Y - 1) / VT_Y));
    k_vanka_sweep<2, FORM, false, T, RS><<<nb, VT_X * VT_Y, 0, s>>>(g, Gp, qp, uo, Ap, ui);
  }
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

bool fused_sweep_ok(int dim, int form, int shape) {
  return dim == 2 && (form == SM_FULL || form == SM_POINT || form == SM_BOX2 ||
                      form == SM_ELEMENT || form == 6 /* symmetric half */) &&
         (shape == CROSS || shape == BOX1 || shape == BOX2);
}

hipError_t vanka_sweep_fused(int dim, int form, int shape, Grid g, int prec, const void* G,
                             double w, const void* A, const void* q, const void* u_in, void* u_out,
                             hipStream_t s) {
  if (!fused_sweep_ok(dim, form, shape) || u_in == u_out) return hipErrorInvalidValue;
  if (form == 6) {
    if (g.Np >= (1LL << 31)) return hipErrorInvalidValue;
#define VH_FS(RS, T)                                                                           \
  if (shape == RS) {                                                                           \
    constexpr int TY = sym_ty<T>();                                                            \
    const unsigned nb = (unsigned)(((g.nx + VT_X - 1) / VT_X) * ((g.ny + TY - 1) / TY));       \
    k_vanka_sweep_sym<2, false, T, RS><<<nb, VT_X * TY, 0, s>>>(                                \
        g, (const cpx<T>*)G, w, (const cpx<T>*)q, (cpx<T>*)u_out, (const cpx<T>*)A,             \
        (const cpx<T>*)u_in);                                                                   \
    VH_LAUNCH_CHECK();                                                                          \
    return hipSuccess;                                                                          \
  }
    if (prec == PREC_F64) {
      VH_FS(CROSS, double) VH_FS(BOX1, double) VH_FS(BOX2, double)
    } else {
      VH_FS(CROSS, float) VH_FS(BOX1, float) VH_FS(BOX2, float)
    }
#undef VH_FS
    return hipErrorInvalidValue;
  }
#define VH_FV(F, RS)                                                                          \
  if (form == F && shape == RS)                                                               \
    return prec == PREC_F64 ? fused_sweep_t<F, RS, double>(g, G, A, q, u_in, u_out, s)       \
                            : fused_sweep_t<F, RS, float>(g, G, A, q, u_in, u_out, s);
  VH_FV(SM_FULL, CROSS) VH_FV(SM_FULL, BOX1) VH_FV(SM_FULL, BOX2)
  VH_FV(SM_POINT, CROSS) VH_FV(SM_POINT, BOX1) VH_FV(SM_POINT, BOX2)
  VH_FV(SM_BOX2, CROSS) VH_FV(SM_BOX2, BOX1) VH_FV(SM_BOX2, BOX2)
  VH_FV(SM_ELEMENT, CROSS) VH_FV(SM_ELEMENT, BOX1) VH_FV(SM_ELEMENT, BOX2)
#undef VH_FV
  return hipErrorInvalidValue;
}

// Assembled form of the same operator: B[d][i] = sum over (a, m) with
// off_m - off_a = d of G[(a*Np+m)][i]  (d in the 5^DIM box, FULL patch), summed
// in FP64.  u += B r is then a 5^DIM-point stencil sweep.
// member index of the offset (mx, my, mz) from the anchor, or -1, in closed form
// (same order as patch_member: 3^DIM-box order for Full, Plus and RB, 2^DIM-box order
// for Element)
template <int DIM, int PATCH>
__device__ __forceinline__ int member_of(int mx, int my, int mz) {
  if (PATCH == PATCH_ELEMENT) {
    if (mx < 0 || mx > 1 || my < 0 || my > 1 || mz < 0 || mz > (DIM == 3 ? 1 : 0)) return -1;
    return mx + 2 * my + 4 * mz;
  }
  if (mx < -1 || mx > 1 || my < -1 || my > 1 || mz < (DIM == 3 ? -1 : 0) || mz > (DIM == 3 ? 1 : 0))
    return -1;
  const int t = (mx + 1) + 3 * (my + 1) + (DIM == 3 ? 9 * (mz + 1) : 0);
  if (PATCH == PATCH_FULL) return t;
  if (!box_member<DIM, PATCH>(t)) return -1;
  int k = 0;  // members of the box before t
  for (int q = 0; q < t; ++q) k += box_member<DIM, PATCH>(q) ? 1 : 0;
  return k;
}

// SYM: only the entries e >= C (C the centre) are formed, as S = B / D (row i divided
// by w / cnt_i), for the symmetric sweep above.
template <int DIM, int PATCH, class T, bool SYM>
__global__ __launch_bounds__(256) void k_vanka_assemble(Grid g, const cpx<T>* __restrict__ G,
                                                        Slab sl, double w, cpx<T>* __restrict__ B) {
  const long long i = sl.c_lo + (long long)node_id();
  if (i >= sl.c_hi) return;
  constexpr int Np = patch_Np<DIM, PATCH>();
  constexpr int K5 = shape_K<DIM, BOX2>();
  const size_t N = (size_t)g.Np;
  int cx, cy, cz;
  decode((unsigned)i, g, cx, cy, cz);
  const long long ip = linp(g, cx, cy, cz);
  const size_t ig = (size_t)(ip - sl.gbase);
  // entry e of the box collects every (a, m) with off_m - off_a = off_e; both loops are
  // unrolled, so the member lookups fold to constants and only existing pairs are loaded
  constexpr int E0 = SYM ? (K5 - 1) / 2 : 0;
  const double rs = SYM ? (double)patch_count<DIM, PATCH>(g, cx, cy, cz) / w : 1.0;
#pragma unroll
  for (int e = E0; e < K5; ++e) {
    const int dx = shape_off<DIM, BOX2>(e, 0), dy = shape_off<DIM, BOX2>(e, 1),
              dz = shape_off<DIM, BOX2>(e, 2);
    cpx<double> acc = cmk(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < Np; ++a) {
      const int m = member_of<DIM, PATCH>(dx + patch_off<DIM, PATCH>(a, 0),
                                          dy + patch_off<DIM, PATCH>(a, 1),
                                          dz + patch_off<DIM, PATCH>(a, 2));
      // rows of patches that do not exist (anchor outside the grid) were never written
      if (m >= 0 && anchor_ok<DIM, PATCH>(g, cx - patch_off<DIM, PATCH>(a, 0),
                                          cy - patch_off<DIM, PATCH>(a, 1),
                                          cz - patch_off<DIM, PATCH>(a, 2)))
        acc = acc + ccast<double>(G[(size_t)(a * Np + m) * sl.gstride + ig]);
    }
    B[(size_t)(e - E0) * N + ip] = ccast<T>(SYM ? rs * acc : acc);
  }
}

template <int PATCH, bool SYM>
static hipError_t assemble_p(int dim, Grid g, int prec, const void* G, Slab sl, double w, void* B,
                             hipStream_t s) {
  const unsigned nb = nblocks((size_t)(sl.c_hi - sl.c_lo), 256);
  if (dim == 2) {
    if (prec == PREC_F64)
      k_vanka_assemble<2, PATCH, double, SYM><<<nb, 256, 0, s>>>(g, (const cpx<double>*)G, sl, w,
                                                                 (cpx<double>*)B);
    else
      k_vanka_assemble<2, PATCH, float, SYM><<<nb, 256, 0, s>>>(g, (const cpx<float>*)G, sl, w,
                                                                (cpx<float>*)B);
  } else {
    if (prec == PREC_F64)
      k_vanka_assemble<3, PATCH, double, SYM><<<nb, 256, 0, s>>>(g, (const cpx<double>*)G, sl, w,
                                                                 (cpx<double>*)B);
    else
      k_vanka_assemble<3, PATCH, float, SYM><<<nb, 256, 0, s>>>(g, (const cpx<float>*)G, sl, w,
                                                                (cpx<float>*)B);
  }
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t vanka_assemble(int dim, int patch, Grid g, int prec, const void* G, Slab sl, void* B,
                          hipStream_t s) {
  if (sl.c_lo < 0 || sl.c_hi > (long long)g.N || sl.c_lo >= sl.c_hi) return hipErrorInvalidValue;
  switch (patch) {
    case PATCH_FULL: return assemble_p<PATCH_FULL, false>(dim, g, prec, G, sl, 1.0, B, s);
    case PATCH_PLUS: return assemble_p<PATCH_PLUS, false>(dim, g, prec, G, sl, 1.0, B, s);
    case PATCH_RB: return assemble_p<PATCH_RB, false>(dim, g, prec, G, sl, 1.0, B, s);
    case PATCH_ELEMENT: return assemble_p<PATCH_ELEMENT, false>(dim, g, prec, G, sl, 1.0, B, s);
    default: return hipErrorInvalidValue;
  }
}

// the upper half of the assembled Full-patch stencil divided by the weights (w > 0)
hipError_t vanka_assemble_sym(int dim, Grid g, int prec, const void* G, Slab sl, double w, void* S,
                              hipStream_t s) {
  if (sl.c_lo < 0 || sl.c_hi > (long long)g.N || sl.c_lo >= sl.c_hi || !(w > 0))
    return hipErrorInvalidValue;
  return assemble_p<PATCH_FULL, true>(dim, g, prec, G, sl, w, S, s);
}

// dst[e][i] (FP64, N-node rows, e over the whole 5^DIM box) = B[e][i] = D_i S(i, i + d_e)
// rebuilt from the stored half: S[e-C][i] for e >= C, S[C'-C][i+d_e] (C' = K5-1-e, the
// mirrored entry stored at i + d_e) for e < C.
__device__ __forceinline__ cpx<double> sym_entry(const Grid& g, int K5, double w, int x, int y, int z,
                                                 int e, const void* S, int prec) {
  const int C = (K5 - 1) / 2;
  const int dx = e % 5 - 2, dy = (e / 5) % 5 - 2, dz = g.dim == 3 ? e / 25 - 2 : 0;
  int q, jx = x, jy = y, jz = z;
  if (e >= C) {
    q = e - C;
  } else {
    q = (K5 - 1 - e) - C;
    jx += dx;
    jy += dy;
    jz += dz;
    if (!inside(g, jx, jy, jz)) return cmk(0.0, 0.0);
  }
  const size_t at = (size_t)q * (size_t)g.Np + (size_t)linp(g, jx, jy, jz);
  const cpx<double> v = prec == PREC_F64 ? ((const cpx<double>*)S)[at]
                                         : ccast<double>(((const cpx<float>*)S)[at]);
  int cnt = (3 - (x == 0) - (x == g.nx - 1)) * (3 - (y == 0) - (y == g.ny - 1));
  if (g.dim == 3) cnt *= 3 - (z == 0) - (z == g.nz - 1);
  return (w / (double)cnt) * v;
}

__global__ __launch_bounds__(256) void k_unpad_sym(Grid g, int K5, double w, int prec, const void* S,
                                                   cpx<double>* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)K5 * (size_t)g.N) return;
  const int e = (int)(t / (size_t)g.N);
  int x, y, z;
  decode((unsigned)(t % (size_t)g.N), g, x, y, z);
  dst[t] = sym_entry(g, K5, w, x, y, z, e, S, prec);
}

hipError_t unpad_sym(Grid g, double w, int prec, const void* S, cpx<double>* dst, hipStream_t s) {
  const int K5 = g.dim == 3 ? 125 : 25;
  const size_t n = (size_t)K5 * (size_t)g.N;
  k_unpad_sym<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, K5, w, prec, S, dst);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

__global__ __launch_bounds__(256) void k_sample_sym(Grid g, int K5, double w, int prec, int count,
                                                    const long long* __restrict__ nodes,
                                                    const void* S, cpx<double>* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)count * K5) return;
  const int k = (int)(t / K5), e = (int)(t % K5);
  int x, y, z;
  decode((unsigned)nodes[k], g, x, y, z);
  out[t] = sym_entry(g, K5, w, x, y, z, e, S, prec);
}

hipError_t sample_sym(Grid g, double w, int prec, int count, const long long* nodes, const void* S,
                      cpx<double>* out, hipStream_t s) {
  const int K5 = g.dim == 3 ? 125 : 25;
  const unsigned nb = (unsigned)(((long long)count * K5 + 255) / 256);
  k_sample_sym<<<nb, 256, 0, s>>>(g, K5, w, prec, count, nodes, S, out);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// dst[e][i] (FP64, N-node rows) = src[e][padded i] (smoother arrays, for inspection)
template <class T>
__global__ __launch_bounds__(256) void k_unpad(Grid g, int E, const cpx<T>* __restrict__ src,
                                               cpx<double>* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)E * (size_t)g.N) return;
  const size_t e = t / (size_t)g.N;
  const unsigned i = (unsigned)(t % (size_t)g.N);
  int x, y, z;
  decode(i, g, x, y, z);
  dst[t] = ccast<double>(src[e * (size_t)g.Np + (size_t)linp(g, x, y, z)]);
}

hipError_t unpad(Grid g, int E, int prec, const void* src, cpx<double>* dst, hipStream_t s) {
  const size_t n = (size_t)E * (size_t)g.N;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (prec == PREC_F64)
    k_unpad<double><<<nb, 256, 0, s>>>(g, E, (const cpx<double>*)src, dst);
  else
    k_unpad<float><<<nb, 256, 0, s>>>(g, E, (const cpx<float>*)src, dst);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// out[k][e] (FP64) = src[e][node_k] for sampled nodes (padded or plain row layout)
template <class T>
__global__ __launch_bounds__(256) void k_sample(Grid g, int E, int padded, int count,
                                                const long long* __restrict__ nodes,
                                                const cpx<T>* __restrict__ src,
                                                cpx<double>* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)count * E) return;
  const int k = (int)(t / E), e = (int)(t % E);
  const long long i = nodes[k];
  int x, y, z;
  decode((unsigned)i, g, x, y, z);
  const size_t col = padded ? (size_t)linp(g, x, y, z) : (size_t)i;
  const size_t ld = padded ? (size_t)g.Np : (size_t)g.N;
  out[t] = ccast<double>(src[(size_t)e * ld + col]);
}

hipError_t sample(Grid g, int E, int padded, int prec, int count, const long long* nodes,
                  const void* src, cpx<double>* out, hipStream_t s) {
  const unsigned nb = (unsigned)(((long long)count * E + 255) / 256);
  if (prec == PREC_F64)
    k_sample<double><<<nb, 256, 0, s>>>(g, E, padded, count, nodes, (const cpx<double>*)src, out);
  else
    k_sample<float><<<nb, 256, 0, s>>>(g, E, padded, count, nodes, (const cpx<float>*)src, out);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------ Galerkin
// Sec. 3.1: H_c = R H P, one thread per coarse node I:
//   H_c[I][J-I] = sum_t r(t) sum_s H[2I+t][s] p(2I+t+off_s - 2J),
// t over the restriction box, s over the fine stencil, J over the coarse box; the
// tensor-product weights are compile-time constants after unrolling.  Terms whose
// fine node 2I+t or coarse node J lie outside the grid are dropped (truncated R, P).
template <int DIM, int SIN, int SOUT, int RF, int PF>
__global__ __launch_bounds__(256) void k_galerkin(Grid gf, Grid gc, const cpx<double>* __restrict__ Af,
                                                  cpx<double>* __restrict__ Ac) {
  const unsigned I = node_id();
  if (I >= gc.N) return;
  int Ix, Iy, Iz;
  decode(I, gc, Ix, Iy, Iz);
  constexpr int KI = shape_K<DIM, SIN>();
  constexpr int KO = shape_K<DIM, SOUT>();
  constexpr int RR = fam_radius(RF);
  constexpr int RW = 2 * RR + 1;
  constexpr int NT = ipow(RW, DIM);
  constexpr int RO = shape_radius<DIM, SOUT>();
  const size_t Nf = (size_t)gf.N;
  cpx<double> acc[KO];
#pragma unroll
  for (int e = 0; e < KO; ++e) acc[e] = cmk(0.0, 0.0);
  bool jok[KO];
#pragma unroll
  for (int e = 0; e < KO; ++e)
    jok[e] = inside(gc, Ix + shape_off<DIM, SOUT>(e, 0), Iy + shape_off<DIM, SOUT>(e, 1),
                    Iz + shape_off<DIM, SOUT>(e, 2));
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tx = t % RW - RR, ty = (t / RW) % RW - RR, tz = (DIM == 3) ? t / (RW * RW) - RR : 0;
    const int fx = 2 * Ix + tx, fy = 2 * Iy + ty, fz = 2 * Iz + tz;
    if (!inside(gf, fx, fy, fz)) continue;
    const double wr = fam_r(RF, tx) * fam_r(RF, ty) * (DIM == 3 ? fam_r(RF, tz) : 1.0);
    const long long fi = lin(gf, fx, fy, fz);
#pragma unroll
    for (int s = 0; s < KI; ++s) {
      const int sx = shape_off<DIM, SIN>(s, 0), sy = shape_off<DIM, SIN>(s, 1),
                sz = shape_off<DIM, SIN>(s, 2);
      const cpx<double> hv = wr * Af[(size_t)s * Nf + fi];
#pragma unroll
      for (int e = 0; e < KO; ++e) {
        const int ex = shape_off<DIM, SOUT>(e, 0), ey = shape_off<DIM, SOUT>(e, 1),
                  ez = shape_off<DIM, SOUT>(e, 2);
        // fine node j = 2I + t + s, coarse node J = I + e: 1D offsets j - 2J
        const int ux = tx + sx - 2 * ex, uy = ty + sy - 2 * ey, uz = tz + sz - 2 * ez;
        const double wp = fam_p(PF, ux) * fam_p(PF, uy) * (DIM == 3 ? fam_p(PF, uz) : 1.0);
        if (wp != 0.0 && jok[e]) acc[e] = cfma(cmk(wp, 0.0), hv, acc[e]);
      }
    }
  }
  (void)RO;
  const size_t Nc = (size_t)gc.N;
#pragma unroll
  for (int e = 0; e < KO; ++e) Ac[(size_t)e * Nc + I] = acc[e];
}

// The same contraction with one thread per (coarse node, output entry e): for coarse
// grids too small to fill the GPU with one thread per node (each such thread runs the
// whole unrolled contraction alone).  The t and s loops, the weights and the order of
// accumulation per entry are those of k_galerkin, so the results are identical; only the
// zero prolongation weights are skipped at run time instead of at compile time.
template <int DIM, int SIN, int SOUT, int RF, int PF>
__global__ __launch_bounds__(256) void k_galerkin_e(Grid gf, Grid gc, const cpx<double>* __restrict__ Af,
                                                    cpx<double>* __restrict__ Ac) {
  const unsigned I = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = (int)blockIdx.y;
  if (I >= gc.N) return;
  int Ix, Iy, Iz;
  decode(I, gc, Ix, Iy, Iz);
  constexpr int KI = shape_K<DIM, SIN>();
  constexpr int RR = fam_radius(RF);
  constexpr int RW = 2 * RR + 1;
  constexpr int NT = ipow(RW, DIM);
  constexpr int RO = shape_radius<DIM, SOUT>();
  constexpr int WO = 2 * RO + 1;
  const int ex = e % WO - RO, ey = (e / WO) % WO - RO, ez = (DIM == 3) ? e / (WO * WO) - RO : 0;
  const size_t Nf = (size_t)gf.N, Nc = (size_t)gc.N;
  cpx<double> acc = cmk(0.0, 0.0);
  if (inside(gc, Ix + ex, Iy + ey, Iz + ez)) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int tx = t % RW - RR, ty = (t / RW) % RW - RR, tz = (DIM == 3) ? t / (RW * RW) - RR : 0;
      const int fx = 2 * Ix + tx, fy = 2 * Iy + ty, fz = 2 * Iz + tz;
      if (!inside(gf, fx, fy, fz)) continue;
      const double wr = fam_r(RF, tx) * fam_r(RF, ty) * (DIM == 3 ? fam_r(RF, tz) : 1.0);
      const long long fi = lin(gf, fx, fy, fz);
#pragma unroll
      for (int q = 0; q < KI; ++q) {
        const int sx = shape_off<DIM, SIN>(q, 0), sy = shape_off<DIM, SIN>(q, 1),
                  sz = shape_off<DIM, SIN>(q, 2);
        const int ux = tx + sx - 2 * ex, uy = ty + sy - 2 * ey, uz = tz + sz - 2 * ez;
        const double wp = fam_p(PF, ux) * fam_p(PF, uy) * (DIM == 3 ? fam_p(PF, uz) : 1.0);
        if (wp != 0.0) {
          const cpx<double> hv = wr * Af[(size_t)q * Nf + fi];
          acc = cfma(cmk(wp, 0.0), hv, acc);
        }
      }
    }
  }
  Ac[(size_t)e * Nc + I] = acc;
}

hipError_t galerkin(int dim, int sin, int sout, int rf, int pf, Grid gf, Grid gc,
                    const cpx<double>* Af, cpx<double>* Ac, hipStream_t s) {
  const unsigned nb = nblocks(gc.N, 256);
  // one thread per node while that fills the GPU; below, one per (node, output entry)
  const bool per_entry = gc.N < (1LL << 19);
#define VH_GK(D, SI, SO, R, P)                                                         \
  if (dim == D && sin == SI && sout == SO && rf == R && pf == P) {                     \
    if (per_entry)                                                                     \
      k_galerkin_e<D, SI, SO, R, P>                                                    \
          <<<dim3(nb, (unsigned)shape_K<D, SO>()), 256, 0, s>>>(gf, gc, Af, Ac);       \
    else                                                                               \
      k_galerkin<D, SI, SO, R, P><<<nb, 256, 0, s>>>(gf, gc, Af, Ac);                  \
    VH_LAUNCH_CHECK();                                                                 \
    return hipSuccess;                                                                 \
  }
  VH_GK(2, CROSS, BOX2, FAM_CUBIC, FAM_CUBIC)   // level-dependent, finest -> 2nd
  VH_GK(2, CROSS, BOX2, FAM_LINEAR, FAM_CUBIC)  // mixed from the finest level
  VH_GK(2, BOX2, BOX2, FAM_LINEAR, FAM_CUBIC)   // level-dependent / mixed below
  VH_GK(2, BOX2, BOX3, FAM_CUBIC, FAM_CUBIC)    // cubic on every level: 7x7 below
  VH_GK(2, BOX3, BOX3, FAM_CUBIC, FAM_CUBIC)
  VH_GK(2, BOX1, BOX2, FAM_CUBIC, FAM_CUBIC)    // compact fine level: level-dependent
  VH_GK(2, BOX1, BOX2, FAM_LINEAR, FAM_CUBIC)   // compact fine level: mixed
  VH_GK(2, CROSS, BOX1, FAM_LINEAR, FAM_LINEAR) // bilinear
  VH_GK(2, BOX1, BOX1, FAM_LINEAR, FAM_LINEAR)
  VH_GK(3, CROSS, BOX1, FAM_LINEAR, FAM_LINEAR) // trilinear
  VH_GK(3, BOX1, BOX1, FAM_LINEAR, FAM_LINEAR)
#undef VH_GK
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ restriction / prolongation
template <int DIM, int RF, class T>
__global__ __launch_bounds__(256) void k_restrict(Grid gf, Grid gc, const cpx<T>* __restrict__ r,
                                                  cpx<T>* __restrict__ rc) {
  const unsigned I = node_id();
  if (I >= gc.N) return;
  int Ix, Iy, Iz;
  decode(I, gc, Ix, Iy, Iz);
  constexpr int RR = fam_radius(RF), RW = 2 * RR + 1, NT = ipow(RW, DIM);
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tx = t % RW - RR, ty = (t / RW) % RW - RR, tz = (DIM == 3) ? t / (RW * RW) - RR : 0;
    const int fx = 2 * Ix + tx, fy = 2 * Iy + ty, fz = 2 * Iz + tz;
    if (inside(gf, fx, fy, fz)) {
      const T w = (T)(fam_r(RF, tx) * fam_r(RF, ty) * (DIM == 3 ? fam_r(RF, tz) : 1.0));
      acc = cfma(cmk<T>(w, 0), r[lin(gf, fx, fy, fz)], acc);
    }
  }
  rc[I] = acc;
}

// u = u_in + P e; u_in is u itself for the in-place correction
template <int DIM, int PF, class T>
__global__ __launch_bounds__(256) void k_prolong_add(Grid gf, Grid gc, const cpx<T>* __restrict__ e,
                                                     cpx<T>* u, const cpx<T>* u_in) {
  const unsigned i = node_id();
  if (i >= gf.N) return;
  int c[3];
  decode(i, gf, c[0], c[1], c[2]);
  if constexpr (PF == FAM_LINEAR) {
    // p(0) = 1, p(+-1) = 1/2: an even index takes coarse node c/2, an odd one the mean of
    // (c-1)/2 and (c+1)/2 (inside, since every fine grid has 2 n_c - 1 nodes).  All 2^DIM
    // candidates are loaded unconditionally; an even index repeats its node with weight 0.
    int ja[3], jb[3];
    T wa[3], wb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool odd = d < DIM && (c[d] & 1);
      ja[d] = c[d] >> 1;
      jb[d] = odd ? ja[d] + 1 : ja[d];
      wa[d] = odd ? (T)0.5 : (T)1;
      wb[d] = odd ? (T)0.5 : (T)0;
    }
    cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
    for (int sz = 0; sz < (DIM == 3 ? 2 : 1); ++sz)
#pragma unroll
      for (int sy = 0; sy < 2; ++sy)
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          const T wt = (sx ? wb[0] : wa[0]) * (sy ? wb[1] : wa[1]) *
                       (DIM == 3 ? (sz ? wb[2] : wa[2]) : (T)1);
          const cpx<T> ev = e[lin(gc, sx ? jb[0] : ja[0], sy ? jb[1] : ja[1],
                                  DIM == 3 ? (sz ? jb[2] : ja[2]) : 0)];
          acc.re = fma(wt, ev.re, acc.re);
          acc.im = fma(wt, ev.im, acc.im);
        }
    u[i] = u_in[i] + acc;
    return;
  }
  // per dimension: candidate coarse nodes J0-1, J0, J0+1 (J0 = c/2) and weights p(c - 2J)
  int J[3][3];
  T w[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int J0 = c[d] >> 1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      J[d][q] = J0 + q - 1;
      w[d][q] = (T)fam_p(PF, c[d] - 2 * (J0 + q - 1));
    }
  }
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
  for (int qz = 0; qz < (DIM == 3 ? 3 : 1); ++qz)
#pragma unroll
    for (int qy = 0; qy < 3; ++qy)
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        const int Jx = J[0][qx], Jy = J[1][qy], Jz = (DIM == 3) ? J[2][qz] : 0;
        const T wt = w[0][qx] * w[1][qy] * (DIM == 3 ? w[2][qz] : (T)1);
        if (wt != (T)0 && inside(gc, Jx, Jy, Jz))
          acc = cfma(cmk<T>(wt, 0), e[lin(gc, Jx, Jy, Jz)], acc);
      }
  u[i] = u_in[i] + acc;
}

hipError_t restrict_(int dim, int rf, Grid gf, Grid gc, int prec, const void* r, void* rc,
                     hipStream_t s) {
  const unsigned nb = nblocks(gc.N, 256);
#define VH_RS(D, R, T)                                                                        \
  if (dim == D && rf == R) {                                                                  \
    k_restrict<D, R, T><<<nb, 256, 0, s>>>(gf, gc, (const cpx<T>*)r, (cpx<T>*)rc);            \
    VH_LAUNCH_CHECK();                                                                        \
    return hipSuccess;                                                                        \
  }
  if (prec == PREC_F64) {
    VH_RS(2, FAM_LINEAR, double) VH_RS(2, FAM_CUBIC, double)
    VH_RS(3, FAM_LINEAR, double) VH_RS(3, FAM_CUBIC, double)
  } else {
    VH_RS(2, FAM_LINEAR, float) VH_RS(2, FAM_CUBIC, float)
    VH_RS(3, FAM_LINEAR, float) VH_RS(3, FAM_CUBIC, float)
  }
#undef VH_RS
  return hipErrorInvalidValue;
}

// rc = R (q - A u) without storing the fine residual.  One block per 64 x 4 tile of
// coarse nodes (one coarse plane in 3D): the fine residual over the tile's footprint (its
// fine nodes plus the transfer radius, about 1.1x the fine nodes it covers in 2D, 1.7x
// in 3D) is formed once into LDS with the arithmetic of the residual sweep, then every
// lane gathers its coarse node in the order of k_restrict, so the result has the bits of
// the two-launch path.
constexpr int RT_X = 64, RT_Y = 4;

template <int DIM, int RF, int SHAPE, class T>
__global__ __launch_bounds__(256) void k_resid_restrict(Grid gf, Grid gc,
                                                        const cpx<T>* __restrict__ A,
                                                        const cpx<T>* __restrict__ q,
                                                        const cpx<T>* __restrict__ u,
                                                        cpx<T>* __restrict__ rc) {
  constexpr int RR = fam_radius(RF), RW = 2 * RR + 1, NT = ipow(RW, DIM);
  constexpr int FX = 2 * RT_X + 2 * RR - 1, FY = 2 * RT_Y + 2 * RR - 1;
  constexpr int FZ = (DIM == 3) ? RW : 1;
  constexpr int NTL = FX * FY * FZ, NPT = (NTL + RT_X * RT_Y - 1) / (RT_X * RT_Y);
  __shared__ cpx<T> tile[NTL];
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (gc.nx + RT_X - 1) / RT_X, nby = (gc.ny + RT_Y - 1) / RT_Y;
  const int bx = (int)(b % (unsigned)nbx), by = (int)((b / (unsigned)nbx) % (unsigned)nby);
  const int bz = (int)(b / (unsigned)(nbx * nby));
  const int X0 = bx * RT_X, Y0 = by * RT_Y, Z0 = bz;
  const int fx0 = 2 * X0 - RR, fy0 = 2 * Y0 - RR, fz0 = (DIM == 3) ? 2 * Z0 - RR : 0;
#pragma unroll 1
  for (int k = 0; k < NPT; ++k) {
    const int e = (int)threadIdx.x + RT_X * RT_Y * k;
    const int tx = e % FX, ty = (e / FX) % FY, tz = e / (FX * FY);
    const int gx = fx0 + tx, gy = fy0 + ty, gz = fz0 + tz;
    const cpx<T> v = resid_tile<DIM, SHAPE, T>(gf, A, q, u, e < NTL, gx, gy, gz);
    if (e < NTL) tile[e] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const int Ix = X0 + (int)threadIdx.x % RT_X, Iy = Y0 + (int)threadIdx.x / RT_X, Iz = Z0;
  if (Ix >= gc.nx || Iy >= gc.ny) return;
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tx = t % RW - RR, ty = (t / RW) % RW - RR, tz = (DIM == 3) ? t / (RW * RW) - RR : 0;
    const int fx = 2 * Ix + tx, fy = 2 * Iy + ty, fz = 2 * Iz + tz;
    if (inside(gf, fx, fy, fz)) {
      const T w = (T)(fam_r(RF, tx) * fam_r(RF, ty) * (DIM == 3 ? fam_r(RF, tz) : 1.0));
      acc = cfma(cmk<T>(w, 0), tile[((fz - fz0) * FY + (fy - fy0)) * FX + (fx - fx0)], acc);
    }
  }
  rc[lin(gc, Ix, Iy, Iz)] = acc;
}

bool fused_restrict_ok(int dim, int rf, int shape) {
  if (dim == 2) return shape == CROSS || shape == BOX1 || shape == BOX2;
  return dim == 3 && rf == FAM_LINEAR && (shape == CROSS || shape == BOX1);
}

hipError_t resid_restrict(int dim, int rf, int shape, Grid gf, Grid gc, int prec, const void* A,
                          const void* q, const void* u, void* rc, hipStream_t s) {
  if (!fused_restrict_ok(dim, rf, shape)) return hipErrorInvalidValue;
  const unsigned nb =
      (unsigned)(((gc.nx + RT_X - 1) / RT_X) * ((gc.ny + RT_Y - 1) / RT_Y) * gc.nz);
#define VH_RR(D, R, S, T)                                                                    \
  if (dim == D && rf == R && shape == S) {                                                   \
    k_resid_restrict<D, R, S, T><<<nb, RT_X * RT_Y, 0, s>>>(                                  \
        gf, gc, (const cpx<T>*)A, (const cpx<T>*)q, (const cpx<T>*)u, (cpx<T>*)rc);          \
    VH_LAUNCH_CHECK();                                                                        \
    return hipSuccess;                                                                        \
  }
#define VH_RR2(T)                                                                             \
  VH_RR(2, FAM_LINEAR, CROSS, T) VH_RR(2, FAM_LINEAR, BOX1, T) VH_RR(2, FAM_LINEAR, BOX2, T)  \
  VH_RR(2, FAM_CUBIC, CROSS, T) VH_RR(2, FAM_CUBIC, BOX1, T) VH_RR(2, FAM_CUBIC, BOX2, T)     \
  VH_RR(3, FAM_LINEAR, CROSS, T) VH_RR(3, FAM_LINEAR, BOX1, T)
  if (prec == PREC_F64) {
    VH_RR2(double)
  } else {
    VH_RR2(float)
  }
#undef VH_RR2
#undef VH_RR
  return hipErrorInvalidValue;
}

// Linear prolongation with two fine nodes per thread, x = 2J and 2J + 1: both take the
// coarse nodes J and J + 1 of their y-z neighbourhood (the even one with weights 1 and 0),
// so each coarse value is loaded once for the pair and the pair's two inputs and outputs
// are adjacent.  The products and their order are those of k_prolong_add, so the results
// are the same bits.
template <int DIM, class T>
__global__ __launch_bounds__(256) void k_prolong_add_lin2(Grid gf, Grid gc,
                                                          const cpx<T>* __restrict__ e,
                                                          cpx<T>* u, const cpx<T>* u_in) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nt = (long long)gc.nx * gf.ny * gf.nz;
  if (t >= nt) return;
  const int J = (int)(t % gc.nx);
  const long long yz = t / gc.nx;
  const int y = (int)(yz % gf.ny), z = (int)(yz / gf.ny);
  const bool odd_y = (y & 1) != 0, odd_z = DIM == 3 && (z & 1) != 0;
  const int ya = y >> 1, yb = odd_y ? ya + 1 : ya, za = z >> 1, zb = odd_z ? za + 1 : za;
  const T wya = odd_y ? (T)0.5 : (T)1, wyb = odd_y ? (T)0.5 : (T)0;
  const T wza = odd_z ? (T)0.5 : (T)1, wzb = odd_z ? (T)0.5 : (T)0;
  const bool pair = 2 * J + 1 < gf.nx;  // the last even node has no odd partner
  cpx<T> a0 = cmk<T>(0, 0), a1 = cmk<T>(0, 0);
#pragma unroll
  for (int sz = 0; sz < (DIM == 3 ? 2 : 1); ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      const T wy = sy ? wyb : wya, wz = DIM == 3 ? (sz ? wzb : wza) : (T)1;
      const int cy = sy ? yb : ya, cz = DIM == 3 ? (sz ? zb : za) : 0;
      const cpx<T> e0 = e[lin(gc, J, cy, cz)];
      const cpx<T> e1 = pair ? e[lin(gc, J + 1, cy, cz)] : e0;
      // even node: weights 1 and 0 in x, both on coarse node J
      const T w0 = ((T)1 * wy) * wz, w0b = ((T)0 * wy) * wz;
      a0.re = fma(w0, e0.re, a0.re);
      a0.im = fma(w0, e0.im, a0.im);
      a0.re = fma(w0b, e0.re, a0.re);
      a0.im = fma(w0b, e0.im, a0.im);
      // odd node: weight 1/2 on J and on J + 1
      const T w1 = ((T)0.5 * wy) * wz;
      a1.re = fma(w1, e0.re, a1.re);
      a1.im = fma(w1, e0.im, a1.im);
      a1.re = fma(w1, e1.re, a1.re);
      a1.im = fma(w1, e1.im, a1.im);
    }
  const long long i = lin(gf, 2 * J, y, z);
  u[i] = u_in[i] + a0;
  if (pair) u[i + 1] = u_in[i + 1] + a1;
}

hipError_t prolong_add(int dim, int pf, Grid gf, Grid gc, int prec, const void* e, void* u,
                       hipStream_t s, const void* u_in) {
  const unsigned nb = nblocks(gf.N, 256);
  if (!u_in) u_in = u;
#define VH_PA(D, P, T)                                                                         \
  if (dim == D && pf == P) {                                                                   \
    k_prolong_add<D, P, T><<<nb, 256, 0, s>>>(gf, gc, (const cpx<T>*)e, (cpx<T>*)u,            \
                                              (const cpx<T>*)u_in);                            \
    VH_LAUNCH_CHECK();                                                                         \
    return hipSuccess;                                                                         \
  }
#define VH_PL(D, T)                                                                            \
  if (dim == D && pf == FAM_LINEAR) {                                                          \
    const long long nt = (long long)gc.nx * gf.ny * gf.nz;                                     \
    k_prolong_add_lin2<D, T><<<nblocks(nt, 256), 256, 0, s>>>(gf, gc, (const cpx<T>*)e,        \
                                                              (cpx<T>*)u, (const cpx<T>*)u_in); \
    VH_LAUNCH_CHECK();                                                                         \
    return hipSuccess;                                                                         \
  }
  if (prec == PREC_F64) {
    VH_PL(2, double) VH_PA(2, FAM_CUBIC, double)
    VH_PL(3, double) VH_PA(3, FAM_CUBIC, double)
  } else {
    VH_PL(2, float) VH_PA(2, FAM_CUBIC, float)
    VH_PL(3, float) VH_PA(3, FAM_CUBIC, float)
  }
#undef VH_PA
#undef VH_PL
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ coarsest grid
// Dense FP64 copy of the coarsest operator, then an in-place Gauss-Jordan inverse
// with partial pivoting (explicit row swaps, columns unscrambled in reverse order).
template <int DIM, int SHAPE>
__global__ __launch_bounds__(256) void k_dense_assemble(Grid g, const cpx<double>* __restrict__ A,
                                                        cpx<double>* __restrict__ D) {
  const unsigned i = node_id();
  if (i >= g.N) return;
  int cx, cy, cz;
  decode(i, g, cx, cy, cz);
  constexpr int K = shape_K<DIM, SHAPE>();
  const size_t N = (size_t)g.N;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int dx = shape_off<DIM, SHAPE>(k, 0), dy = shape_off<DIM, SHAPE>(k, 1),
              dz = shape_off<DIM, SHAPE>(k, 2);
    if (inside(g, cx + dx, cy + dy, cz + dz)) {
      const long long j = lin(g, cx + dx, cy + dy, cz + dz);
      D[(size_t)i * N + j] = A[(size_t)k * N + i];
    }
  }
}

hipError_t dense_assemble(int dim, int shape, Grid g, const cpx<double>* A, cpx<double>* D,
                          hipStream_t s) {
  const unsigned nb = nblocks(g.N, 256);
#define VH_DA(DD, S)                                                   \
  if (dim == DD && shape == S) {                                       \
    k_dense_assemble<DD, S><<<nb, 256, 0, s>>>(g, A, D);               \
    VH_LAUNCH_CHECK();                                                 \
    return hipSuccess;                                                 \
  }
  VH_DA(2, CROSS) VH_DA(2, BOX1) VH_DA(2, BOX2) VH_DA(2, BOX3) VH_DA(3, CROSS) VH_DA(3, BOX1)
  VH_DA(3, BOX2)
#undef VH_DA
  return hipErrorInvalidValue;
}

// pivot search in column k (rows >= k), row swap, scaling of the pivot row, and a
// copy of column k (zero at the pivot row) for the elimination kernel
__global__ __launch_bounds__(256) void k_gj_pivot(int n, int k, cpx<double>* __restrict__ M,
                                                  int* __restrict__ perm,
                                                  cpx<double>* __restrict__ col) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int t = threadIdx.x;
  double bv = -1.0;
  int bi = k;
  for (int r = k + t; r < n; r += 256) {
    const cpx<double> v = M[(size_t)r * n + k];
    const double a = fabs(v.re) + fabs(v.im);
    if (a > bv) {
      bv = a;
      bi = r;
    }
  }
  sv[t] = bv;
  si[t] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      const double ov = sv[t + w];
      const int oi = si[t + w];
      if (ov > sv[t] || (ov == sv[t] && oi < si[t])) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  if (t == 0) perm[k] = p;
  if (p != k) {
    for (int j = t; j < n; j += 256) {
      const cpx<double> a = M[(size_t)k * n + j];
      M[(size_t)k * n + j] = M[(size_t)p * n + j];
      M[(size_t)p * n + j] = a;
    }
  }
  __syncthreads();
  const cpx<double> inv = cinv(M[(size_t)k * n + k]);
  __syncthreads();
  for (int j = t; j < n; j += 256) {
    const cpx<double> a = (j == k) ? cmk(1.0, 0.0) : M[(size_t)k * n + j];
    M[(size_t)k * n + j] = a * inv;
  }
  for (int r = t; r < n; r += 256) col[r] = (r == k) ? cmk(0.0, 0.0) : M[(size_t)r * n + k];
}

__global__ __launch_bounds__(256) void k_gj_elim(int n, int k, cpx<double>* __restrict__ M,
                                                 const cpx<double>* __restrict__ col) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= n || r == k) return;
  const cpx<double> f = col[r];
  if (f.re == 0.0 && f.im == 0.0) return;
  const cpx<double> pk = M[(size_t)k * n + j];
  if (j == k)
    M[(size_t)r * n + k] = cmk(0.0, 0.0) - f * pk;
  else
    M[(size_t)r * n + j] = M[(size_t)r * n + j] - f * pk;
}

__global__ __launch_bounds__(256) void k_gj_unscramble(int n, cpx<double>* __restrict__ M,
                                                       const int* __restrict__ perm) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {
      const cpx<double> a = M[(size_t)r * n + k];
      M[(size_t)r * n + k] = M[(size_t)r * n + p];
      M[(size_t)r * n + p] = a;
    }
  }
}

// Blocked form of the same elimination: b pivot steps at a time.  One workgroup takes a
// panel of b columns into LDS together with the b identity columns the steps introduce
// (column k of the identity enters at step k, after that step's row swap), and runs the b
// steps there: pivot search in the panel column, row swap, scaling of the pivot row,
// elimination of every other row.  The identity columns end up holding the panel's
// columns of the in-place inverse, Ip (n x b).  Every other column x of the matrix takes
// the same b steps at once: the swaps permute its rows (x -> x[sig]) and the scalings and
// eliminations add Ip - E times its values at the panel rows (E the panel's unit
// columns), since each step reads x only at its pivot row.  So one panel launch and one
// update launch replace 2b launches, with the pivots of the unblocked elimination.
constexpr int GJ_PANEL_MAX = 32;
constexpr int GJ_LDS_ENTRIES = 8960;   // n * 2b complex FP64 entries (140 KB)
constexpr int GJ_MAX_N = 2400;         // rows of the blocked form (row map in LDS)

int gj_panel(int n) {
  const int b = GJ_LDS_ENTRIES / (2 * (n > 0 ? n : 1));
  return (n > GJ_MAX_N || b < 2) ? 0 : (b > GJ_PANEL_MAX ? GJ_PANEL_MAX : b);
}

static size_t gj_align(size_t x) { return (x + 255) / 256 * 256; }

size_t gj_workspace_bytes(int n) {
  const size_t nn = (size_t)n;
  const int b = gj_panel(n);
  if (b == 0) return gj_align(nn * sizeof(int)) + gj_align(nn * sizeof(cpx<double>));
  return gj_align(nn * sizeof(int)) * 2 + gj_align(nn * nn * sizeof(cpx<double>)) +
         gj_align(nn * (size_t)b * sizeof(cpx<double>));
}

__global__ __launch_bounds__(1024) void k_gj_panel(int n, int k0, int b,
                                                   const cpx<double>* __restrict__ M,
                                                   int* __restrict__ perm, int* __restrict__ sig,
                                                   cpx<double>* __restrict__ Ip) {
  __shared__ cpx<double> P[GJ_LDS_ENTRIES];  // [n][2b]: panel columns, then identity columns
  __shared__ int rmap[GJ_MAX_N];             // row of the panel's input now at each row
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ int spiv;
  const int t = threadIdx.x, W2 = 2 * b;
  for (int e = t; e < n * W2; e += 1024) {
    const int r = e / W2, c = e % W2;
    P[e] = c < b ? M[(size_t)r * n + k0 + c] : cmk(0.0, 0.0);
  }
  for (int r = t; r < n; r += 1024) rmap[r] = r;
  __syncthreads();
  for (int tt = 0; tt < b; ++tt) {
    const int k = k0 + tt;
    // pivot: the largest |re| + |im| in the panel column at rows >= k (the first on ties)
    double bv = -1.0;
    int bi = k;
    for (int r = k + t; r < n; r += 1024) {
      const cpx<double> v = P[r * W2 + tt];
      const double a = fabs(v.re) + fabs(v.im);
      if (a > bv) {
        bv = a;
        bi = r;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_down(bv, o, 64);
      const int oi = __shfl_down(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if ((t & 63) == 0) {
      sv[t >> 6] = bv;
      si[t >> 6] = bi;
    }
    __syncthreads();
    if (t == 0) {
      double v = sv[0];
      int i = si[0];
      for (int w = 1; w < 16; ++w)
        if (sv[w] > v || (sv[w] == v && si[w] < i)) {
          v = sv[w];
          i = si[w];
        }
      spiv = i;
      perm[k] = i;
      const int m = rmap[k];
      rmap[k] = rmap[i];
      rmap[i] = m;
    }
    __syncthreads();
    const int p = spiv;
    if (p != k && t < W2) {
      const cpx<double> a = P[k * W2 + t];
      P[k * W2 + t] = P[p * W2 + t];
      P[p * W2 + t] = a;
    }
    __syncthreads();
    if (t == 0) P[k * W2 + b + tt] = cmk(1.0, 0.0);  // identity column k, after the swap
    __syncthreads();
    // scale the pivot row (the pivot column itself is dropped: it becomes a unit column)
    const cpx<double> inv = cinv(P[k * W2 + tt]);
    __syncthreads();
    if (t > tt && t <= b + tt) P[k * W2 + t] = P[k * W2 + t] * inv;
    __syncthreads();
    // eliminate the pivot column from every other row: the remaining panel columns and
    // the identity columns introduced so far
    const int cols = b;  // columns tt+1 .. b+tt
    for (int e = t; e < n * cols; e += 1024) {
      const int r = e / cols, c = tt + 1 + e % cols;
      if (r == k) continue;
      const cpx<double> f = P[r * W2 + tt];
      P[r * W2 + c] = P[r * W2 + c] - f * P[k * W2 + c];
    }
    __syncthreads();
  }
  for (int e = t; e < n * b; e += 1024) Ip[e] = P[(e / b) * W2 + b + e % b];
  for (int r = t; r < n; r += 1024) sig[r] = rmap[r];
}

// Md = the matrix after the panel's steps: the panel's columns from Ip; every other
// column j: x[sig] (panel rows excluded) + Ip x[sig[panel rows]]
constexpr int GJU_ROWS = 16;
__global__ __launch_bounds__(256) void k_gj_update(int n, int k0, int b,
                                                   const cpx<double>* __restrict__ Ms,
                                                   cpx<double>* __restrict__ Md,
                                                   const int* __restrict__ sig,
                                                   const cpx<double>* __restrict__ Ip) {
  __shared__ cpx<double> yp[GJ_PANEL_MAX][64];
  const int jj = threadIdx.x & 63;
  const int j = blockIdx.x * 64 + jj;
  for (int e = threadIdx.x; e < b * 64; e += 256) {
    const int q = e >> 6, jg = blockIdx.x * 64 + (e & 63);
    yp[q][e & 63] = jg < n ? Ms[(size_t)sig[k0 + q] * n + jg] : cmk(0.0, 0.0);
  }
  __syncthreads();
  if (j >= n) return;
  const int r1 = min(n, (int)(blockIdx.y + 1) * GJU_ROWS);
  for (int r = blockIdx.y * GJU_ROWS + (int)(threadIdx.x >> 6); r < r1; r += 4) {
    cpx<double> out;
    if (j >= k0 && j < k0 + b) {
      out = Ip[(size_t)r * b + (j - k0)];
    } else {
      const bool prow = r >= k0 && r < k0 + b;
      cpx<double> acc = prow ? cmk(0.0, 0.0) : Ms[(size_t)sig[r] * n + j];
      for (int q = 0; q < b; ++q) acc = cfma(Ip[(size_t)r * b + q], yp[q][jj], acc);
      out = acc;
    }
    Md[(size_t)r * n + j] = out;
  }
}

hipError_t gj_invert(int n, cpx<double>* M, void* work, hipStream_t s) {
  char* w = (char*)work;
  int* perm = (int*)w;
  const int b = gj_panel(n);
  if (b == 0) {  // one pivot step per launch pair
    cpx<double>* col = (cpx<double>*)(w + gj_align((size_t)n * sizeof(int)));
    for (int k = 0; k < n; ++k) {
      k_gj_pivot<<<1, 256, 0, s>>>(n, k, M, perm, col);
      VH_LAUNCH_CHECK();
      dim3 grid((n + 255) / 256, n);
      k_gj_elim<<<grid, 256, 0, s>>>(n, k, M, col);
      VH_LAUNCH_CHECK();
    }
  } else {
    int* sig = (int*)(w + gj_align((size_t)n * sizeof(int)));
    cpx<double>* M2 = (cpx<double>*)(w + 2 * gj_align((size_t)n * sizeof(int)));
    cpx<double>* Ip = (cpx<double>*)((char*)M2 + gj_align((size_t)n * n * sizeof(cpx<double>)));
    cpx<double>* cur = M;
    cpx<double>* oth = M2;
    const dim3 ug((unsigned)((n + 63) / 64), (unsigned)((n + GJU_ROWS - 1) / GJU_ROWS));
    for (int k0 = 0; k0 < n; k0 += b) {
      const int bb = (n - k0) < b ? (n - k0) : b;
      k_gj_panel<<<1, 1024, 0, s>>>(n, k0, bb, cur, perm, sig, Ip);
      VH_LAUNCH_CHECK();
      k_gj_update<<<ug, 256, 0, s>>>(n, k0, bb, cur, oth, sig, Ip);
      VH_LAUNCH_CHECK();
      cpx<double>* tmp = cur;
      cur = oth;
      oth = tmp;
    }
    if (cur != M) {
      const hipError_t e =
          hipMemcpyAsync(M, cur, (size_t)n * n * sizeof(cpx<double>), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
  }
  k_gj_unscramble<<<(n + 255) / 256, 256, 0, s>>>(n, M, perm);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// y = D x with D the FP64 dense inverse; one wavefront per row, fixed-order reduction
template <class T>
__global__ __launch_bounds__(256) void k_dense_matvec(int n, const cpx<double>* __restrict__ D,
                                                      const cpx<T>* __restrict__ x,
                                                      cpx<T>* __restrict__ y) {
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  cpx<double> acc = cmk(0.0, 0.0);
  for (int j = lane; j < n; j += 64) acc = cfma(D[(size_t)row * n + j], ccast<double>(x[j]), acc);
  for (int o = 32; o > 0; o >>= 1) {
    acc.re += __shfl_down(acc.re, o, 64);
    acc.im += __shfl_down(acc.im, o, 64);
  }
  if (lane == 0) y[row] = ccast<T>(acc);
}

hipError_t dense_matvec(int n, const cpx<double>* D, int prec, const void* x, void* y,
                        hipStream_t s) {
  const unsigned nb = (unsigned)((n * 64 + 255) / 256);
  if (prec == PREC_F64)
    k_dense_matvec<double><<<nb, 256, 0, s>>>(n, D, (const cpx<double>*)x, (cpx<double>*)y);
  else
    k_dense_matvec<float><<<nb, 256, 0, s>>>(n, D, (const cpx<float>*)x, (cpx<float>*)y);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------ Krylov (FP64)
// Block-partial multi-dot: part[b][j] = sum over block b's chunk of conj(V_j) w,
// j < nv (nv <= KMAX).  Chunks are contiguous, partials are reduced in block order.
constexpr int KMAX = 65;

__device__ __forceinline__ cpx<double> wave_sum(cpx<double> v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_down(v.re, o, 64);
    v.im += __shfl_down(v.im, o, 64);
  }
  return v;
}

// block reduction of one complex value, result valid in thread 0
__device__ __forceinline__ cpx<double> block_sum(cpx<double> v, cpx<double>* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  cpx<double> out = cmk(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) out = out + sh[q];
  return out;
}

__device__ __forceinline__ void chunk(size_t N, size_t& lo, size_t& hi) {
  const size_t per = (N + gridDim.x - 1) / gridDim.x;
  lo = (size_t)blockIdx.x * per;
  hi = lo + per < N ? lo + per : N;
}

// mode 0: part = V^H w;  mode 1: w -= V h, part = V^H w (after the update);
// mode 2: w -= V h, part[0] = ||w||^2.
template <int MODE>
__global__ __launch_bounds__(256) void k_cgs(const cpx<double>* __restrict__ V, size_t ldv, int nv,
                                             const cpx<double>* __restrict__ h,
                                             cpx<double>* __restrict__ w, size_t N,
                                             cpx<double>* __restrict__ part) {
  __shared__ cpx<double> sh[4];
  __shared__ cpx<double> hs[KMAX];
  if (MODE != 0) {
    for (int j = threadIdx.x; j < nv; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
  }
  size_t lo, hi;
  chunk(N, lo, hi);
  const int nout = (MODE == 2) ? 1 : nv;
  // process the outputs in groups of 8 to bound register use
  for (int j0 = 0; j0 < nout; j0 += 8) {
    cpx<double> acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = cmk(0.0, 0.0);
    for (size_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      cpx<double> wi = w[i];
      if (MODE != 0 && j0 == 0) {
        for (int j = 0; j < nv; ++j) wi = wi - hs[j] * V[(size_t)j * ldv + i];
        w[i] = wi;
      }
      if (MODE == 2) {
        acc[0].re += wi.re * wi.re + wi.im * wi.im;
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (j0 + q < nv) acc[q] = cfma_conj(V[(size_t)(j0 + q) * ldv + i], wi, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (j0 + q < nout) {
        const cpx<double> s = block_sum(acc[q], sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * KMAX + j0 + q] = s;
      }
    }
    if (MODE != 0) __syncthreads();
  }
}

// out[j] = sum_b part[b][j]: one block per output, fixed-order strided sums then a
// fixed-order tree (bitwise reproducible)
__global__ __launch_bounds__(256) void k_reduce_part(const cpx<double>* __restrict__ part, int nb,
                                                     cpx<double>* __restrict__ out) {
  __shared__ cpx<double> sh[256];
  const int j = blockIdx.x, t = threadIdx.x;
  cpx<double> s = cmk(0.0, 0.0);
  for (int b = t; b < nb; b += 256) s = s + part[(size_t)b * KMAX + j];
  sh[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  if (t == 0) out[j] = sh[0];
}

// Register-resident form of k_cgs for nv <= 8 * P: P lanes per node, lane q of a node
// holding columns 8q .. 8q + 7 (one accumulator each), nodes dealt to the lane groups
// of the grid round-robin.  A pass reads each column of V once and w once; in MODE 1
// the column values loaded for the update are reused for the new dot products.  The
// update w - V h is summed over the P lanes of a node by a butterfly, which leaves the
// same bits in every lane.  Columns j >= nv re-read column nv - 1 with a zero
// coefficient and their sums are discarded, so every load is unconditional.
template <int MODE, int P>
__global__ __launch_bounds__(256) void k_cgs_r(const cpx<double>* __restrict__ V, size_t ldv,
                                               int nv, const cpx<double>* __restrict__ h,
                                               cpx<double>* __restrict__ w, size_t N,
                                               cpx<double>* __restrict__ part) {
  constexpr int CJ = 8, NJ = CJ * P;
  constexpr int NA = (MODE == 2) ? 1 : CJ;
  __shared__ cpx<double> red[4][64];
  __shared__ cpx<double> hs[NJ];
  if (MODE != 0) {
    if (threadIdx.x < NJ) hs[threadIdx.x] = (int)threadIdx.x < nv ? h[threadIdx.x] : cmk(0.0, 0.0);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane % P;  // column group of this lane
  const size_t slot = ((size_t)blockIdx.x * 256 + threadIdx.x) / P;
  const size_t stride = (size_t)gridDim.x * (256 / P);
  int col[CJ];
#pragma unroll
  for (int c = 0; c < CJ; ++c) col[c] = (q * CJ + c < nv) ? q * CJ + c : (nv > 0 ? nv - 1 : 0);
  cpx<double> acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c) acc[c] = cmk(0.0, 0.0);
  for (size_t i = slot; i < N; i += stride) {
    cpx<double> wi = w[i];
    cpx<double> v[CJ];
    if (MODE == 0 || nv > 0) {  // the norm-only pass at a restart has nv == 0
#pragma unroll
      for (int c = 0; c < CJ; ++c) v[c] = V[(size_t)col[c] * ldv + i];
    }
    if (MODE != 0 && nv > 0) {
      cpx<double> t = cmk(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < CJ; ++c) t = cfma(hs[q * CJ + c], v[c], t);
#pragma unroll
      for (int o = 1; o < P; o <<= 1) {
        t.re += __shfl_xor(t.re, o, 64);
        t.im += __shfl_xor(t.im, o, 64);
      }
      wi = wi - t;
      if (q == 0) w[i] = wi;
    }
    if (MODE == 2) {
      if (q == 0) acc[0].re += wi.re * wi.re + wi.im * wi.im;
    } else {
#pragma unroll
      for (int c = 0; c < CJ; ++c) acc[c] = cfma_conj(v[c], wi, acc[c]);
    }
  }
  // lanes with the same q hold sums of the same columns: fold them (stride P within
  // the wavefront), then the four wavefronts; column q*CJ + c ends in part[b][.]
  const int nout = (MODE == 2) ? 1 : nv;
#pragma unroll
  for (int c = 0; c < NA; ++c) {
    if (c < nout) {  // uniform over the block
      cpx<double> x = acc[c];
      for (int o = 32; o >= P; o >>= 1) {
        x.re += __shfl_down(x.re, o, 64);
        x.im += __shfl_down(x.im, o, 64);
      }
      __syncthreads();
      if (lane < P) red[wv][lane] = x;
      __syncthreads();
      if (threadIdx.x < P) {
        const int j = (int)threadIdx.x * CJ + c;
        if (j < nout) {
          cpx<double> t = red[0][threadIdx.x];
          for (int k = 1; k < 4; ++k) t = t + red[k][threadIdx.x];
          part[(size_t)blockIdx.x * KMAX + j] = t;
        }
      }
    }
  }
}

// Blocks of 256 threads resident at once on the whole device for kernel k (queried
// once per kernel; every device the library runs on is the same gfx950 part).
template <class Kern>
static int resident_blocks(Kern k) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 256, 0) != hipSuccess || per < 1)
    return 1 << 30;
  return per * ncu;
}

// one pass on a grid of at most one resident wave of blocks; returns the partial rows
template <int MODE, int P>
static int cgs_r(const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h, cpx<double>* w,
                 size_t N, cpx<double>* part, int nb, hipStream_t s) {
  static const int res = resident_blocks(k_cgs_r<MODE, P>);
  const int g = nb < res ? nb : res;
  k_cgs_r<MODE, P><<<g, 256, 0, s>>>(V, ldv, nv, h, w, N, part);
  return g;
}

template <int MODE>
static int cgs_launch(const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                      cpx<double>* w, size_t N, cpx<double>* part, int nb, hipStream_t s) {
  if (nv <= 8) return cgs_r<MODE, 1>(V, ldv, nv, h, w, N, part, nb, s);
  if (nv <= 16) return cgs_r<MODE, 2>(V, ldv, nv, h, w, N, part, nb, s);
  if (nv <= 32) return cgs_r<MODE, 4>(V, ldv, nv, h, w, N, part, nb, s);
  if (nv <= 64) return cgs_r<MODE, 8>(V, ldv, nv, h, w, N, part, nb, s);
  k_cgs<MODE><<<nb, 256, 0, s>>>(V, ldv, nv, h, w, N, part);
  return nb;
}

hipError_t cgs_pass(int mode, const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                    cpx<double>* w, size_t N, cpx<double>* part, int nb, cpx<double>* out,
                    hipStream_t s) {
  if (nv < (mode == 2 ? 0 : 1) || nv > KMAX) return hipErrorInvalidValue;
  int rows;
  if (mode == 0)
    rows = cgs_launch<0>(V, ldv, nv, h, w, N, part, nb, s);
  else if (mode == 1)
    rows = cgs_launch<1>(V, ldv, nv, h, w, N, part, nb, s);
  else
    rows = cgs_launch<2>(V, ldv, nv, h, w, N, part, nb, s);
  VH_LAUNCH_CHECK();
  k_reduce_part<<<mode == 2 ? 1 : nv, 256, 0, s>>>(part, rows, out);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// Arnoldi column j: H[:,j] = h1 + h2 (CGS2), H[j+1][j] = ||w||; apply the previous
// Givens rotations, form the new one, update g; status = |g[j+1]|, 1/||w||.
__global__ void k_arnoldi_finalize(KrylovDev* __restrict__ K, int j, int ldh) {
  if (threadIdx.x != 0) return;
  cpx<double>* Hc = K->H + (size_t)j * ldh;
  for (int i = 0; i <= j; ++i) Hc[i] = K->h1[i] + K->h2[i];
  const double nrm = sqrt(K->nrm2[0].re);
  Hc[j + 1] = cmk(nrm, 0.0);
  for (int i = 0; i < j; ++i) {
    const cpx<double> a = Hc[i], b = Hc[i + 1];
    const double c = K->cs[i];
    const cpx<double> sn = K->sn[i];
    Hc[i] = c * a + sn * b;
    Hc[i + 1] = c * b - cmk(sn.re, -sn.im) * a;
  }
  const cpx<double> a = Hc[j];
  const double b = nrm;
  double c;
  cpx<double> sn;
  const double aa = sqrt(a.re * a.re + a.im * a.im);
  if (aa == 0.0) {
    c = 0.0;
    sn = cmk(1.0, 0.0);
  } else {
    const double r = sqrt(aa * aa + b * b);
    c = aa / r;
    sn = cmk(a.re / aa * b / r, a.im / aa * b / r);  // (a/|a|) * conj(b) / r, b real
  }
  K->cs[j] = c;
  K->sn[j] = sn;
  Hc[j] = c * a + sn * cmk(b, 0.0);
  Hc[j + 1] = cmk(0.0, 0.0);
  const cpx<double> gj = K->g[j];
  K->g[j + 1] = cmk(0.0, 0.0) - cmk(sn.re, -sn.im) * gj;
  K->g[j] = c * gj;
  const cpx<double> gn = K->g[j + 1];
  K->status[0] = sqrt(gn.re * gn.re + gn.im * gn.im);
  K->status[1] = nrm;
  K->inv_nrm = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  const bool bad = !(nrm == nrm) || !(K->status[0] == K->status[0]) || isinf(nrm);
  K->status[2] = bad ? 1.0 : 0.0;
}

hipError_t arnoldi_finalize(KrylovDev* K, int j, int ldh, hipStream_t s) {
  k_arnoldi_finalize<<<1, 64, 0, s>>>(K, j, ldh);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// y = R^{-1} g (k x k upper triangle of H)
__global__ void k_backsolve(KrylovDev* __restrict__ K, int k, int ldh) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    cpx<double> s = K->g[i];
    for (int q = i + 1; q < k; ++q) s = s - K->H[(size_t)q * ldh + i] * K->y[q];
    K->y[i] = s * cinv(K->H[(size_t)i * ldh + i]);
  }
}

hipError_t backsolve(KrylovDev* K, int k, int ldh, hipStream_t s) {
  k_backsolve<<<1, 64, 0, s>>>(K, k, ldh);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// x += sum_j y_j Z_j  (Z at the preconditioner precision)
template <class TZ>
__global__ __launch_bounds__(256) void k_update_x(const KrylovDev* __restrict__ K, int k,
                                                  const cpx<TZ>* __restrict__ Z, size_t ldz,
                                                  cpx<double>* __restrict__ x, size_t N) {
  __shared__ cpx<double> ys[KMAX];
  for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = K->y[j];
  __syncthreads();
  const size_t i = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  cpx<double> a = x[i];
  for (int j = 0; j < k; ++j) a = cfma(ys[j], ccast<double>(Z[(size_t)j * ldz + i]), a);
  x[i] = a;
}

hipError_t update_x(const KrylovDev* K, int k, int pz, const void* Z, size_t ldz,
                    cpx<double>* x, size_t N, hipStream_t s) {
  const unsigned nb = nblocks((long long)N, 256);
  if (pz == PREC_F64)
    k_update_x<double><<<nb, 256, 0, s>>>(K, k, (const cpx<double>*)Z, ldz, x, N);
  else
    k_update_x<float><<<nb, 256, 0, s>>>(K, k, (const cpx<float>*)Z, ldz, x, N);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// v = w * scale (scale read from the device: K->inv_nrm or 1/beta)
__global__ __launch_bounds__(256) void k_scale(const double* __restrict__ scale,
                                               const cpx<double>* __restrict__ w,
                                               cpx<double>* __restrict__ v, size_t N) {
  const size_t i = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  v[i] = scale[0] * w[i];
}

hipError_t scale_vec(const double* scale, const cpx<double>* w, cpx<double>* v, size_t N,
                     hipStream_t s) {
  k_scale<<<nblocks((long long)N, 256), 256, 0, s>>>(scale, w, v, N);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

// new cycle: beta = sqrt(nrm2), inv_nrm = 1/beta, g = (beta, 0, ...)
__global__ void k_cycle_init(KrylovDev* __restrict__ K, int m) {
  if (threadIdx.x != 0) return;
  const double beta = sqrt(K->nrm2[0].re);
  K->g[0] = cmk(beta, 0.0);
  for (int i = 1; i <= m; ++i) K->g[i] = cmk(0.0, 0.0);
  K->inv_nrm = beta > 0.0 ? 1.0 / beta : 0.0;
  K->status[3] = beta;
}

hipError_t cycle_init(KrylovDev* K, int m, hipStream_t s) {
  k_cycle_init<<<1, 64, 0, s>>>(K, m);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace vh
