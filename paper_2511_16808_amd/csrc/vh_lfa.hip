// vh_lfa.hip -- local Fourier analysis of the Vanka smoothers and of the two-grid cycle
// on the device (Sec. 2.4, Sec. 4), and the LFA damping tuner of Sec. 5.2.
//
// The operator is the interior stencil A of H_s for constant sigma = omega^2 kappa^2:
// the 5/7-point stencil or the compact 4th-order stencil (eq. (disc4thCompact),
// (disc4thCompact3D)), with the shift i * shift * M.  For a patch with members o_k:
//   patch matrix     A_i[k][m] = A at offset o_m - o_k,
//   smoother symbol  S(theta) = 1 - w q(theta) A(theta),
//                    q(theta) = phi^H A_i^{-1} phi / Np, phi_k = exp(i theta.o_k)
//                    (eq. (smoother_symbol): every node is in Np patches),
//   two-grid symbol  TG = S^nu2 (I - P H_c^{-1} R A) S^nu1 on the 2^dim harmonics
//                    (eq. (symbolTG)), H_c = sum_h R_h A_h P_h (Galerkin, Sec. 4.2).
// Everything is FP64.  Kernels: the patch inverse (one block), one thread per theta
// sample for q, A, R, P, then one thread per (theta, w) pair for |S| or the spectral
// radius of TG, block maxima, and a last block that reduces them and picks the
// minimiser over w.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vh.h"
#include "vh_launch.h"

using namespace vh;

void vh_internal_set_error(const std::string& msg);  // vh_runtime.hip

namespace {

#define VH_LAUNCH_CHECK()               \
  do {                                  \
    hipError_t e__ = hipGetLastError(); \
    if (e__ != hipSuccess) return e__;  \
  } while (0)

constexpr int LFA_MAXN = 27;  // largest patch: the 3D Full patch
constexpr int LFA_T = 256;    // threads per block of the theta kernels

struct LfaConst {
  cpx<double> st[27];                    // A on the 3^DIM box (x fastest)
  cpx<double> inv[LFA_MAXN * LFA_MAXN];  // A_i^{-1}, row-major
  int singular;
};

__device__ __forceinline__ cpx<double> cdiv(cpx<double> a, cpx<double> b) { return a * cinv(b); }
__device__ __forceinline__ double cabs_(cpx<double> a) { return hypot(a.re, a.im); }

// box index (x fastest) of the offset (dx, dy, dz), each in [-1, 1]
template <int DIM>
__device__ __forceinline__ int box_idx(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
}

// ------------------------------------------------------------------ stencil and patch inverse
template <int DIM, int PATCH>
__global__ __launch_bounds__(64) void k_lfa_prep(int stencil, double h, double sigma, double shift,
                                                  LfaConst* __restrict__ C) {
  constexpr int N = patch_Np<DIM, PATCH>();
  constexpr int NB = ipow(3, DIM);
  __shared__ cpx<double> st[27];
  __shared__ cpx<double> a[N][2 * N];
  const int t = threadIdx.x;
  const double ih2 = 1.0 / (h * h);
  if (t < NB) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
    const int l1 = abs(dx) + abs(dy) + abs(dz);
    cpx<double> v;
    if (stencil == VH_STENCIL_COMPACT4) {
      const double m = compact_M<DIM>(l1);
      v = cmk(compact_L<DIM>(l1, ih2) - sigma * m, shift * m);
    } else {
      v = l1 == 0 ? cmk(2.0 * DIM * ih2 - sigma, shift) : cmk(l1 == 1 ? -ih2 : 0.0, 0.0);
    }
    st[t] = v;
    C->st[t] = v;
  }
  __syncthreads();
  // [A_i | I], then Gauss-Jordan with partial pivoting (one thread: Np <= 27)
  for (int e = t; e < N * 2 * N; e += blockDim.x) {
    const int k = e / (2 * N), m = e % (2 * N);
    cpx<double> v = cmk(0.0, 0.0);
    if (m < N) {
      const int ox = patch_off<DIM, PATCH>(m, 0) - patch_off<DIM, PATCH>(k, 0);
      const int oy = patch_off<DIM, PATCH>(m, 1) - patch_off<DIM, PATCH>(k, 1);
      const int oz = patch_off<DIM, PATCH>(m, 2) - patch_off<DIM, PATCH>(k, 2);
      // members up to 2 apart (Full, Plus, RB) see no coupling beyond the 3^DIM stencil
      if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) v = st[box_idx<DIM>(ox, oy, oz)];
    } else if (m - N == k) {
      v = cmk(1.0, 0.0);
    }
    a[k][m] = v;
  }
  __syncthreads();
  if (t != 0) return;
  int singular = 0;
  for (int c = 0; c < N; ++c) {
    int piv = c;
    double best = cabs_(a[c][c]);
    for (int k = c + 1; k < N; ++k) {
      const double v = cabs_(a[k][c]);
      if (v > best) {
        best = v;
        piv = k;
      }
    }
    if (!(best > 0.0)) {
      singular = 1;
      break;
    }
    if (piv != c)
      for (int m = 0; m < 2 * N; ++m) {
        const cpx<double> s = a[c][m];
        a[c][m] = a[piv][m];
        a[piv][m] = s;
      }
    const cpx<double> ip = cinv(a[c][c]);
    for (int m = 0; m < 2 * N; ++m) a[c][m] = ip * a[c][m];
    for (int k = 0; k < N; ++k) {
      if (k == c) continue;
      const cpx<double> f = a[k][c];
      for (int m = 0; m < 2 * N; ++m) a[k][m] = a[k][m] - f * a[c][m];
    }
  }
  for (int k = 0; k < N; ++k)
    for (int m = 0; m < N; ++m) C->inv[k * N + m] = a[k][N + m];
  C->singular = singular;
}

// ------------------------------------------------------------------ per-theta symbols
__device__ __forceinline__ double theta_of(int k, int npts) {
  return -0.5 * M_PI + 2.0 * M_PI * (double)k / (double)npts;
}

// 1D symbol of the family's weights, sum_t r_t exp(i t th) (real: the weights are even)
__device__ __forceinline__ double fam_symbol(int fam, double th) {
  double s = fam_r(fam, 0);
  for (int t = 1; t <= fam_radius(fam); ++t) s += 2.0 * fam_r(fam, t) * cos(t * th);
  return s;
}

template <int DIM, int PATCH>
__global__ __launch_bounds__(LFA_T) void k_lfa_theta(int npts, int rfam, int pfam, long long count,
                                                     const LfaConst* __restrict__ C,
                                                     cpx<double>* __restrict__ Z,
                                                     cpx<double>* __restrict__ Asym,
                                                     double* __restrict__ Rs,
                                                     double* __restrict__ Ps) {
  constexpr int N = patch_Np<DIM, PATCH>();
  constexpr int NB = ipow(3, DIM);
  __shared__ cpx<double> inv[N * N];
  __shared__ cpx<double> st[NB];
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) inv[e] = C->inv[e];
  for (int e = threadIdx.x; e < NB; e += blockDim.x) st[e] = C->st[e];
  __syncthreads();
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    double th[3] = {0.0, 0.0, 0.0};
    long long r = i;
    for (int d = 0; d < DIM; ++d) {
      th[d] = theta_of((int)(r % npts), npts);
      r /= npts;
    }
    // exp(i th_d o) for o = -1, 0, 1
    cpx<double> e[3][3];
    for (int d = 0; d < 3; ++d) {
      double sn, cs;
      sincos(th[d], &sn, &cs);
      e[d][0] = cmk(cs, -sn);
      e[d][1] = cmk(1.0, 0.0);
      e[d][2] = cmk(cs, sn);
    }
    cpx<double> A = cmk(0.0, 0.0);
    for (int t = 0; t < NB; ++t) {
      const int ox = t % 3, oy = (t / 3) % 3, oz = DIM == 3 ? t / 9 : 1;
      A = cfma(st[t], e[0][ox] * e[1][oy] * e[2][oz], A);
    }
    cpx<double> phi[N];
    for (int k = 0; k < N; ++k)
      phi[k] = e[0][patch_off<DIM, PATCH>(k, 0) + 1] * e[1][patch_off<DIM, PATCH>(k, 1) + 1] *
               e[2][patch_off<DIM, PATCH>(k, 2) + 1];
    cpx<double> q = cmk(0.0, 0.0);
    for (int k = 0; k < N; ++k) {
      cpx<double> row = cmk(0.0, 0.0);
      for (int m = 0; m < N; ++m) row = cfma(inv[k * N + m], phi[m], row);
      q = cfma_conj(phi[k], row, q);
    }
    q = (1.0 / N) * q;
    double R = 1.0, P = 1.0;
    for (int d = 0; d < DIM; ++d) {
      R *= fam_symbol(rfam, th[d]);
      P *= fam_symbol(pfam, th[d]);
    }
    Z[i] = q * A;
    Asym[i] = A;
    Rs[i] = R;
    Ps[i] = P;
  }
}

// block maximum of v (non-negative; NaN propagates) into part[blockIdx.y * gridDim.x + blockIdx.x]
__device__ void block_max(double v, double* __restrict__ part) {
  __shared__ double red[LFA_T];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = LFA_T / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      const double c = red[threadIdx.x];
      red[threadIdx.x] = (o > c || o != o) ? o : c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ smoothing factor
__global__ __launch_bounds__(LFA_T) void k_lfa_mu(int dim, int npts, long long count,
                                                  const cpx<double>* __restrict__ Z,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ part) {
  const double wj = w[blockIdx.y];
  double m = 0.0;
  const int half = npts / 2;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    long long r = i;
    bool high = false;
    for (int d = 0; d < dim; ++d) {
      high |= (int)(r % npts) >= half;  // theta_d >= pi/2
      r /= npts;
    }
    if (!high) continue;
    const cpx<double> z = Z[i];
    const double v = hypot(1.0 - wj * z.re, -wj * z.im);
    m = (v > m || v != v) ? v : m;
  }
  block_max(m, part);
}

// ------------------------------------------------------------------ two-grid factor
// Largest root modulus of the monic polynomial sum_j c_j x^j (c[n] = 1) by the
// Aberth-Ehrlich simultaneous iteration, started on a circle of the radius
// max_j |c_j|^(1/(n-j)); corrections are applied in place (Gauss-Seidel order).
template <int n>
__device__ double max_root(const cpx<double>* c) {
  double R = 0.0;
  for (int j = 0; j < n; ++j) {
    const double a = cabs_(c[j]);
    if (a > 0.0) R = fmax(R, pow(a, 1.0 / (n - j)));
  }
  if (!(R > 0.0)) return R == R ? 0.0 : R;
  cpx<double> z[n];
  for (int k = 0; k < n; ++k) {
    double sn, cs;
    sincos(2.0 * M_PI * k / n + 0.4, &sn, &cs);
    z[k] = cmk(R * cs, R * sn);
  }
  for (int it = 0; it < 300; ++it) {
    double dmax = 0.0;
    for (int k = 0; k < n; ++k) {
      cpx<double> p = c[n], dp = cmk(0.0, 0.0);
      for (int j = n - 1; j >= 0; --j) {
        dp = dp * z[k] + p;
        p = p * z[k] + c[j];
      }
      if (p.re == 0.0 && p.im == 0.0) continue;
      if (dp.re == 0.0 && dp.im == 0.0) dp = cmk(1e-300, 0.0);
      const cpx<double> ratio = cdiv(p, dp);
      cpx<double> s = cmk(0.0, 0.0);
      for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        const cpx<double> d = z[k] - z[j];
        if (d.re != 0.0 || d.im != 0.0) s = s + cinv(d);
      }
      const cpx<double> corr = cdiv(ratio, cmk(1.0, 0.0) - ratio * s);
      z[k] = z[k] - corr;
      dmax = fmax(dmax, cabs_(corr));
    }
    if (!(dmax > 1e-16 * R)) break;
  }
  double m = 0.0;
  for (int k = 0; k < n; ++k) m = fmax(m, cabs_(z[k]));
  return m;
}

// eig(S^nu2 K S^nu1) = eig(K D) with D = diag(S_h^(nu1+nu2)), K = I - p g^T,
// p_h = P_h, g_h = R_h A_h / H_c.  det(x I - D + p (D g)^T)
//   = prod_h (x - d_h) + sum_h p_h g_h d_h prod_{j != h} (x - d_j).
template <int DIM>
__global__ __launch_bounds__(LFA_T) void k_lfa_rho(int npts, int nu, long long count,
                                                   const cpx<double>* __restrict__ Z,
                                                   const cpx<double>* __restrict__ Asym,
                                                   const double* __restrict__ Rs,
                                                   const double* __restrict__ Ps,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ part) {
  constexpr int NH = 1 << DIM;
  const double wj = w[blockIdx.y];
  const int half = npts / 2;
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    int kl[3] = {0, 0, 0};
    long long r = i;
    bool zero = true;
    for (int d = 0; d < DIM; ++d) {
      kl[d] = (int)(r % half);
      r /= half;
      zero &= fabs(theta_of(kl[d], npts)) <= 1e-12;
    }
    if (zero) continue;  // theta = 0: H_c vanishes when sigma = 0
    cpx<double> zh[NH], ah[NH];
    double rh[NH], ph[NH];
    cpx<double> Hc = cmk(0.0, 0.0);
    for (int hb = 0; hb < NH; ++hb) {
      long long idx = 0, stride = 1;
      for (int d = 0; d < DIM; ++d) {
        idx += stride * (kl[d] + (((hb >> d) & 1) ? half : 0));
        stride *= npts;
      }
      zh[hb] = Z[idx];
      ah[hb] = Asym[idx];
      rh[hb] = Rs[idx];
      ph[hb] = Ps[idx];
      Hc = Hc + (rh[hb] * ph[hb]) * ah[hb];
    }
    const cpx<double> iHc = cinv(Hc);
    cpx<double> dh[NH], ch[NH];
    for (int hb = 0; hb < NH; ++hb) {
      const cpx<double> s = cmk(1.0 - wj * zh[hb].re, -wj * zh[hb].im);
      cpx<double> d = cmk(1.0, 0.0);
      for (int k = 0; k < nu; ++k) d = d * s;
      dh[hb] = d;
      ch[hb] = (ph[hb] * rh[hb]) * (ah[hb] * iHc) * d;
    }
    // coefficients, lowest degree first
    cpx<double> c[NH + 1];
    for (int j = 0; j <= NH; ++j) c[j] = cmk(j == 0 ? 1.0 : 0.0, 0.0);
    for (int j = 0; j < NH; ++j) {  // c <- c * (x - d_j), degree j -> j + 1
      for (int t = j + 1; t >= 1; --t) c[t] = c[t - 1] - dh[j] * c[t];
      c[0] = cmk(0.0, 0.0) - dh[j] * c[0];
    }
    for (int hb = 0; hb < NH; ++hb) {
      cpx<double> b[NH];
      for (int j = 0; j < NH; ++j) b[j] = cmk(j == 0 ? 1.0 : 0.0, 0.0);
      int deg = 0;
      for (int j = 0; j < NH; ++j) {
        if (j == hb) continue;
        for (int t = deg + 1; t >= 1; --t) b[t] = b[t - 1] - dh[j] * b[t];
        b[0] = cmk(0.0, 0.0) - dh[j] * b[0];
        ++deg;
      }
      for (int t = 0; t < NH; ++t) c[t] = c[t] + ch[hb] * b[t];
    }
    const double v = max_root<NH>(c);
    m = (v > m || v != v) ? v : m;
  }
  block_max(m, part);
}

// out[j] = max over the nbx block maxima of candidate j; best[0] = index of the first
// minimiser (as a double), best[1] = its value
__global__ __launch_bounds__(256) void k_lfa_final(int nw, int nbx, const double* __restrict__ part,
                                                   double* __restrict__ out,
                                                   double* __restrict__ best) {
  for (int j = threadIdx.x; j < nw; j += blockDim.x) {
    double m = 0.0;
    for (int b = 0; b < nbx; ++b) {
      const double v = part[(size_t)j * nbx + b];
      m = (v > m || v != v) ? v : m;
    }
    out[j] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int bi = -1;
    double bv = 0.0;
    for (int j = 0; j < nw; ++j)
      if (out[j] == out[j] && (bi < 0 || out[j] < bv)) {
        bi = j;
        bv = out[j];
      }
    best[0] = (double)bi;
    best[1] = bi < 0 ? NAN : bv;
  }
}

vh_status lfail(vh_status st, const std::string& m) {
  vh_internal_set_error(m);
  return st;
}

#define LFA_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      st = lfail(VH_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
      goto done;                                                                           \
    }                                                                                      \
  } while (0)

template <int DIM, int PATCH>
hipError_t launch_symbols(const vh_lfa_problem* p, LfaConst* C, long long count, int nbx,
                          cpx<double>* Z, cpx<double>* A, double* R, double* P, hipStream_t s) {
  const int rf = p->rfam == VH_IG_LINEAR ? FAM_LINEAR : FAM_CUBIC;
  const int pf = p->pfam == VH_IG_LINEAR ? FAM_LINEAR : FAM_CUBIC;
  k_lfa_prep<DIM, PATCH><<<1, 64, 0, s>>>(p->stencil, p->h, p->sigma, p->shift, C);
  VH_LAUNCH_CHECK();
  k_lfa_theta<DIM, PATCH><<<nbx, LFA_T, 0, s>>>(p->npts, rf, pf, count, C, Z, A, R, P);
  VH_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t symbols(const vh_lfa_problem* p, LfaConst* C, long long count, int nbx,
                   cpx<double>* Z, cpx<double>* A, double* R, double* P, hipStream_t s) {
#define VH_LS(D, PT) \
  if (p->dim == D && p->patch == PT) return launch_symbols<D, PT>(p, C, count, nbx, Z, A, R, P, s);
  VH_LS(2, PATCH_FULL)
  VH_LS(2, PATCH_POINT)
  VH_LS(2, PATCH_PLUS)
  VH_LS(2, PATCH_RB)
  VH_LS(2, PATCH_ELEMENT)
  VH_LS(3, PATCH_FULL)
  VH_LS(3, PATCH_POINT)
  VH_LS(3, PATCH_PLUS)
  VH_LS(3, PATCH_RB)
  VH_LS(3, PATCH_ELEMENT)
#undef VH_LS
  return hipErrorInvalidValue;
}

vh_status check(const vh_lfa_problem* p, int nw, const double* w) {
  if (!p || !w || nw < 1 || nw > 4096) return lfail(VH_EINVAL, "bad LFA arguments");
  if (p->dim != 2 && p->dim != 3) return lfail(VH_EINVAL, "dim must be 2 or 3");
  if (p->stencil != VH_STENCIL_FD2 && p->stencil != VH_STENCIL_COMPACT4)
    return lfail(VH_EINVAL, "unknown stencil");
  if (p->patch != VH_PATCH_FULL && p->patch != VH_PATCH_POINT && p->patch != VH_PATCH_PLUS &&
      p->patch != VH_PATCH_RB && p->patch != VH_PATCH_ELEMENT)
    return lfail(VH_EINVAL, "unknown patch");
  if (!(p->h > 0.0) || !(p->sigma >= 0.0) || !(p->shift >= 0.0) || !std::isfinite(p->h) ||
      !std::isfinite(p->sigma) || !std::isfinite(p->shift))
    return lfail(VH_EINVAL, "h > 0, sigma >= 0 and shift >= 0 must be finite");
  if ((p->rfam != VH_IG_LINEAR && p->rfam != VH_IG_CUBIC) ||
      (p->pfam != VH_IG_LINEAR && p->pfam != VH_IG_CUBIC))
    return lfail(VH_EINVAL, "rfam and pfam must be VH_IG_LINEAR or VH_IG_CUBIC");
  const int nmax = p->dim == 2 ? 512 : 128;
  if (p->npts < 4 || p->npts > nmax || (p->npts % 2) != 0)
    return lfail(VH_EINVAL, "npts must be even, >= 4 and <= 512 (2D) / 128 (3D)");
  if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 + p->nu2 > 8)
    return lfail(VH_EINVAL, "nu1, nu2 >= 0 with nu1 + nu2 <= 8");
  for (int j = 0; j < nw; ++j)
    if (!std::isfinite(w[j])) return lfail(VH_EINVAL, "non-finite damping");
  return VH_OK;
}

// Placement of the LFA work arrays in one device buffer: the stencil and patch inverse,
// per theta sample q(theta) and A(theta) (complex) and R(theta), P(theta) (real), the
// damping values, the block maxima and the reduced factors.
struct LfaLayout {
  long long count, lcount;  // npts^dim samples, (npts/2)^dim low frequencies
  int nbx, nbl;             // blocks of the per-sample and per-low-frequency kernels
  size_t o_Z, o_A, o_R, o_P, o_w, o_part, o_out, bytes;
};

LfaLayout lfa_layout(const vh_lfa_problem* p, int nw) {
  LfaLayout L;
  L.count = 1;
  for (int d = 0; d < p->dim; ++d) L.count *= p->npts;
  L.lcount = L.count >> p->dim;
  L.nbx = (int)std::min<long long>((L.count + LFA_T - 1) / LFA_T, 256);
  L.nbl = (int)std::min<long long>((L.lcount + LFA_T - 1) / LFA_T, 256);
  L.o_Z = (sizeof(LfaConst) + 255) / 256 * 256;
  L.o_A = L.o_Z + (size_t)L.count * 16;
  L.o_R = L.o_A + (size_t)L.count * 16;
  L.o_P = L.o_R + (size_t)L.count * 8;
  L.o_w = L.o_P + (size_t)L.count * 8;
  L.o_part = L.o_w + (size_t)nw * 8;
  L.o_out = L.o_part + (size_t)nw * std::max(L.nbx, L.nbl) * 8;
  L.bytes = L.o_out + (size_t)(2 * nw + 4) * 8;
  return L;
}

// Enqueues the LFA kernels on p->stream with their arrays in buf (laid out by lfa_layout);
// every array is written before it is read, so buf needs no clearing.  The factors are
// left in buf at o_out: mu[nw], rho[nw], then (index, value) of the minimiser of each.
hipError_t lfa_enqueue(const vh_lfa_problem* p, int nw, const double* w, bool want_mu,
                       bool want_rho, const LfaLayout& L, char* buf) {
  hipStream_t s = (hipStream_t)p->stream;
  LfaConst* C = (LfaConst*)buf;
  double* wd = (double*)(buf + L.o_w);
  double* part = (double*)(buf + L.o_part);
  double* out = (double*)(buf + L.o_out);
  hipError_t e = hipMemcpyAsync(wd, w, (size_t)nw * 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = symbols(p, C, L.count, L.nbx, (cpx<double>*)(buf + L.o_Z), (cpx<double>*)(buf + L.o_A),
              (double*)(buf + L.o_R), (double*)(buf + L.o_P), s);
  if (e != hipSuccess) return e;
  if (want_mu) {
    k_lfa_mu<<<dim3(L.nbx, nw), LFA_T, 0, s>>>(p->dim, p->npts, L.count,
                                               (const cpx<double>*)(buf + L.o_Z), wd, part);
    VH_LAUNCH_CHECK();
    k_lfa_final<<<1, 256, 0, s>>>(nw, L.nbx, part, out, out + 2 * nw);
    VH_LAUNCH_CHECK();
  }
  if (want_rho) {
    const int nu = p->nu1 + p->nu2;
    if (p->dim == 2)
      k_lfa_rho<2><<<dim3(L.nbl, nw), LFA_T, 0, s>>>(
          p->npts, nu, L.lcount, (const cpx<double>*)(buf + L.o_Z),
          (const cpx<double>*)(buf + L.o_A), (const double*)(buf + L.o_R),
          (const double*)(buf + L.o_P), wd, part);
    else
      k_lfa_rho<3><<<dim3(L.nbl, nw), LFA_T, 0, s>>>(
          p->npts, nu, L.lcount, (const cpx<double>*)(buf + L.o_Z),
          (const cpx<double>*)(buf + L.o_A), (const double*)(buf + L.o_R),
          (const double*)(buf + L.o_P), wd, part);
    VH_LAUNCH_CHECK();
    k_lfa_final<<<1, 256, 0, s>>>(nw, L.nbl, part, out + nw, out + 2 * nw + 2);
    VH_LAUNCH_CHECK();
  }
  return hipSuccess;
}

// objective: 0 = mu, 1 = rho; out (host) receives the nw factors of each requested one
vh_status run(const vh_lfa_problem* p, int nw, const double* w, double* mu, double* rho,
              double* best_mu, double* best_rho) {
  vh_status st = check(p, nw, w);
  if (st != VH_OK) return st;
  hipStream_t s = (hipStream_t)p->stream;
  const LfaLayout L = lfa_layout(p, nw);
  char* buf = nullptr;
  double* host = nullptr;
  int singular = 0;
  LFA_HIP(hipMalloc((void**)&buf, L.bytes));
  LFA_HIP(lfa_enqueue(p, nw, w, mu != nullptr, rho != nullptr, L, buf));
  LFA_HIP(hipHostMalloc((void**)&host, (size_t)(2 * nw + 4) * 8, hipHostMallocDefault));
  LFA_HIP(hipMemcpyAsync(host, buf + L.o_out, (size_t)(2 * nw + 4) * 8, hipMemcpyDeviceToHost, s));
  LFA_HIP(hipMemcpyAsync(&singular, &((LfaConst*)buf)->singular, sizeof(int),
                         hipMemcpyDeviceToHost, s));
  LFA_HIP(hipStreamSynchronize(s));
  if (singular) {
    st = lfail(VH_EBREAKDOWN, "the patch matrix of the stencil is singular");
    goto done;
  }
  if (mu) {
    for (int j = 0; j < nw; ++j) mu[j] = host[j];
    if (best_mu) {
      best_mu[0] = host[2 * nw];
      best_mu[1] = host[2 * nw + 1];
    }
  }
  if (rho) {
    for (int j = 0; j < nw; ++j) rho[j] = host[nw + j];
    if (best_rho) {
      best_rho[0] = host[2 * nw + 2];
      best_rho[1] = host[2 * nw + 3];
    }
  }
done:
  if (host) (void)hipHostFree(host);
  if (buf) (void)hipFree(buf);
  return st;
}

// ------------------------------------------------------------------ allocation-free form
// The work arrays of vh_lfa_factors_noalloc live in one statically allocated device array
// per GPU (held until the process ends).  In host code `scratch` names only a host-side
// stand-in: its device address is looked up once per device with hipGetSymbolAddress and
// only that address is handed to copies and kernels.
constexpr size_t LFA_SCRATCH_BYTES = (size_t)16 << 20;
constexpr int LFA_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) char scratch[LFA_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_dev[LFA_MAX_DEVICES] = {};

// device address of the scratch array on the current device (looked up on first use)
vh_status scratch_address(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lfail(VH_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= LFA_MAX_DEVICES) return lfail(VH_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return lfail(VH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (char*)ptr;
  }
  *out = g_scratch_dev[dev];
  return VH_OK;
}

}  // namespace

extern "C" {

void vh_lfa_problem_default(vh_lfa_problem* p) {
  if (!p) return;
  *p = vh_lfa_problem{};
  p->dim = 2;
  p->stencil = VH_STENCIL_FD2;
  p->patch = VH_PATCH_FULL;
  p->h = 1.0 / 256;
  p->sigma = 0.0;
  p->shift = 0.0;
  p->rfam = VH_IG_CUBIC;
  p->pfam = VH_IG_CUBIC;
  p->npts = 256;
  p->nu1 = 1;
  p->nu2 = 1;
  p->stream = nullptr;
}

vh_status vh_lfa_factors(const vh_lfa_problem* p, int nw, const double* w, double* mu,
                         double* rho) {
  if (!mu && !rho) return lfail(VH_EINVAL, "mu and rho are both NULL");
  return run(p, nw, w, mu, rho, nullptr, nullptr);
}

vh_status vh_lfa_factors_noalloc(const vh_lfa_problem* p, int nw, const double* w, double* mu,
                                 double* rho) {
  if (!mu && !rho) return lfail(VH_EINVAL, "mu and rho are both NULL");
  vh_status st = check(p, nw, w);
  if (st != VH_OK) return st;
  const LfaLayout L = lfa_layout(p, nw);
  if (L.bytes > LFA_SCRATCH_BYTES)
    return lfail(VH_EINVAL, "the LFA work arrays need " + std::to_string(L.bytes) +
                                " bytes; the allocation-free form holds at most " +
                                std::to_string(LFA_SCRATCH_BYTES) +
                                " (npts^dim <= 2^18 samples and nw <= 1024)");
  char* buf = nullptr;
  st = scratch_address(&buf);
  if (st != VH_OK) return st;
  hipStream_t s = (hipStream_t)p->stream;
  int singular = 0;
  LFA_HIP(lfa_enqueue(p, nw, w, mu != nullptr, rho != nullptr, L, buf));
  if (mu) LFA_HIP(hipMemcpyAsync(mu, buf + L.o_out, (size_t)nw * 8, hipMemcpyDeviceToHost, s));
  if (rho)
    LFA_HIP(hipMemcpyAsync(rho, buf + L.o_out + (size_t)nw * 8, (size_t)nw * 8,
                           hipMemcpyDeviceToHost, s));
  LFA_HIP(hipMemcpyAsync(&singular, &((LfaConst*)buf)->singular, sizeof(int),
                         hipMemcpyDeviceToHost, s));
  LFA_HIP(hipStreamSynchronize(s));
  if (singular) st = lfail(VH_EBREAKDOWN, "the patch matrix of the stencil is singular");
done:
  return st;
}

vh_status vh_lfa_tune(const vh_lfa_problem* p, int objective, int nw, const double* w,
                      double* w_best, double* f_best) {
  if ((objective != 0 && objective != 1) || !w_best || !f_best)
    return lfail(VH_EINVAL, "objective must be 0 (mu) or 1 (rho); w_best, f_best non-NULL");
  std::vector<double> f((size_t)std::max(nw, 1));
  double best[2] = {-1.0, NAN};
  vh_status st = objective == 0 ? run(p, nw, w, f.data(), nullptr, best, nullptr)
                                : run(p, nw, w, nullptr, f.data(), nullptr, best);
  if (st != VH_OK) return st;
  const int bi = (int)best[0];
  if (bi < 0 || bi >= nw) return lfail(VH_EBREAKDOWN, "every LFA factor is NaN");
  *w_best = w[bi];
  *f_best = best[1];
  return VH_OK;
}

}  // extern "C"
