// vh_common.h -- device types, compile-time stencil shapes and kernel launchers.
//
// Internal header of the gfx950 library; the public ABI is include/vh.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace vh {

// ---------------------------------------------------------------- complex scalars
template <class T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <class T>
__host__ __device__ __forceinline__ cpx<T> cmk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return cmk(a.re + b.re, a.im + b.im);
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return cmk(a.re - b.re, a.im - b.im);
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) {
  return cmk(s * a.re, s * a.im);
}
// acc + a*b with fused multiply-adds
template <class T>
__host__ __device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a)*b
template <class T>
__host__ __device__ __forceinline__ cpx<T> cfma_conj(cpx<T> a, cpx<T> b, cpx<T> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
template <class TO, class TI>
__host__ __device__ __forceinline__ cpx<TO> ccast(cpx<TI> a) {
  return cmk<TO>(static_cast<TO>(a.re), static_cast<TO>(a.im));
}
template <class T>
__host__ __device__ __forceinline__ cpx<T> cinv(cpx<T> a) {
  // 1/a with a scaling step so that |a|^2 does not overflow or underflow
  T s = fmax(fabs(a.re), fabs(a.im));
  T ar = a.re / s, ai = a.im / s;
  T d = ar * ar + ai * ai;
  return cmk<T>(ar / (d * s), -ai / (d * s));
}

// ---------------------------------------------------------------- grids
struct Grid {
  int nx, ny, nz;  // nodes per dimension (nz = 1 in 2D)
  int dim;
  long long N;    // nx*ny*nz
  int nxp;        // x extent of the padded layout used by the smoother arrays
  long long Np;   // nxp*ny*nz
  // off-diagonals of a 5/7-point operator: 0 = read from the coefficient array;
  // 1 (Dirichlet rows) / 2 (absorbing rows) = the fixed values -ih2, -2 ih2 times the
  // boundary scaling, computed in the kernel (only the centre coefficient is read)
  int offrule;
  double ih2;
  double rnx, rnxy;  // 1/nx and 1/(nx*ny) in FP64, for the node decode
};

// Smoother arrays ([entry][node], one row per entry) use rows of nxp = nx rounded up
// to 32 nodes, so that every 64-node run a wavefront loads starts on a cache-line
// boundary whatever nx is.
constexpr int ROW_ALIGN = 32;

__host__ __device__ __forceinline__ Grid make_grid(int dim, int nx, int ny, int nz) {
  Grid g;
  g.nx = nx;
  g.ny = ny;
  g.nz = (dim == 3) ? nz : 1;
  g.dim = dim;
  g.N = (long long)g.nx * g.ny * g.nz;
  g.nxp = (nx + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  g.Np = (long long)g.nxp * g.ny * g.nz;
  g.offrule = 0;
  g.ih2 = 0.0;
  g.rnx = 1.0 / (double)g.nx;
  g.rnxy = 1.0 / ((double)g.nx * (double)g.ny);
  return g;
}

// (x, y, z) of node i < 2^31: each quotient from the FP64 reciprocal (within one of the
// true quotient), then one correction step either way; no integer division
__device__ __forceinline__ void grid_decode(unsigned i, const Grid& g, int& x, int& y, int& z) {
  const unsigned long long nxy = (unsigned long long)g.nx * (unsigned long long)g.ny;
  unsigned zq = (unsigned)((double)i * g.rnxy);
  if ((unsigned long long)zq * nxy > i) --zq;
  if ((unsigned long long)(zq + 1) * nxy <= i) ++zq;
  const unsigned rem = i - (unsigned)((unsigned long long)zq * nxy);
  unsigned yq = (unsigned)((double)rem * g.rnx);
  if (yq * (unsigned)g.nx > rem) --yq;
  if ((yq + 1) * (unsigned)g.nx <= rem) ++yq;
  x = (int)(rem - yq * (unsigned)g.nx);
  y = (int)yq;
  z = (int)zq;
}

// ---------------------------------------------------------------- stencil shapes
// CROSS: centre + the 2*DIM axis neighbours, ordered centre, -x, +x, -y, +y, -z, +z.
// BOX<r>: the (2r+1)^DIM box, x fastest (BOX3 = 7x7: Galerkin operators below the second
// level with cubic restriction and prolongation on every level, 2D only).
enum Shape : int { CROSS = 0, BOX1 = 1, BOX2 = 2, BOX3 = 3 };

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int SHAPE>
__host__ __device__ constexpr int shape_K() {
  return SHAPE == CROSS ? 2 * DIM + 1 : ipow(2 * SHAPE + 1, DIM);
}

template <int DIM, int SHAPE>
__host__ __device__ constexpr int shape_radius() {
  return SHAPE == CROSS ? 1 : SHAPE;
}

// component c (0 = x, 1 = y, 2 = z) of the offset of entry k
template <int DIM, int SHAPE>
__host__ __device__ constexpr int shape_off(int k, int c) {
  if (SHAPE == CROSS) {
    if (k == 0) return 0;
    return ((k - 1) / 2 == c) ? (((k - 1) % 2 == 0) ? -1 : 1) : 0;
  }
  if (c >= DIM) return 0;
  return (k / ipow(2 * SHAPE + 1, c)) % (2 * SHAPE + 1) - SHAPE;
}

// entry index of offset (dx, dy, dz), or -1 if the shape does not contain it
template <int DIM, int SHAPE>
__host__ __device__ constexpr int shape_index(int dx, int dy, int dz) {
  if (DIM == 2 && dz != 0) return -1;
  if (SHAPE == CROSS) {
    int nz = (dx != 0) + (dy != 0) + (dz != 0);
    if (nz == 0) return 0;
    if (nz > 1) return -1;
    if (dx == -1) return 1;
    if (dx == 1) return 2;
    if (dy == -1) return 3;
    if (dy == 1) return 4;
    if (dz == -1) return 5;
    if (dz == 1) return 6;
    return -1;
  }
  const int r = SHAPE, W = 2 * SHAPE + 1;
  if (dx < -r || dx > r || dy < -r || dy > r || dz < -r || dz > r) return -1;
  return (dx + r) + W * (dy + r) + (DIM == 3 ? W * W * (dz + r) : 0);
}

// Vanka patches (Sec. 3.2): FULL = the 3^DIM box; POINT = the node itself; PLUS = the
// node and its 2*DIM axis neighbours; RB = the members of the 3^DIM box with the same
// red-black colour as the centre (|dx| + |dy| + |dz| even); ELEMENT = the 2^DIM corners
// of the cell whose lowest corner is the anchor.  Members of FULL, PLUS and RB are in
// 3^DIM-box order (x fastest), ELEMENT in 2^DIM-box order (x fastest).  Every node
// anchors a (truncated) patch, except for ELEMENT, anchored at every cell only.
// Value 2 is the assembled-stencil form of the sweep, not a patch.
enum Patch : int { PATCH_FULL = 0, PATCH_POINT = 1, PATCH_PLUS = 3, PATCH_RB = 4, PATCH_ELEMENT = 5 };

// does member t of the 3^DIM box (x fastest) belong to the patch?
template <int DIM, int PATCH>
__host__ __device__ constexpr bool box_member(int t) {
  const int ax = t % 3 - 1, ay = (t / 3) % 3 - 1, az = DIM == 3 ? t / 9 - 1 : 0;
  const int l1 = (ax < 0 ? -ax : ax) + (ay < 0 ? -ay : ay) + (az < 0 ? -az : az);
  return PATCH == PATCH_FULL ? true
         : PATCH == PATCH_PLUS ? l1 <= 1
         : PATCH == PATCH_RB   ? (l1 % 2 == 0)
                               : l1 == 0;
}

template <int DIM, int PATCH>
__host__ __device__ constexpr int patch_Np() {
  if (PATCH == PATCH_ELEMENT) return ipow(2, DIM);
  int n = 0;
  for (int t = 0; t < ipow(3, DIM); ++t) n += box_member<DIM, PATCH>(t) ? 1 : 0;
  return n;
}

template <int DIM, int PATCH>
__host__ __device__ constexpr int patch_off(int k, int c) {
  if (c >= DIM) return 0;
  if (PATCH == PATCH_ELEMENT) return (k >> c) & 1;
  int seen = 0;
  for (int t = 0; t < ipow(3, DIM); ++t)
    if (box_member<DIM, PATCH>(t)) {
      if (seen == k) return (t / ipow(3, c)) % 3 - 1;
      ++seen;
    }
  return 0;
}

// index of the member at offset (dx, dy, dz) from the anchor, or -1
template <int DIM, int PATCH>
__host__ __device__ constexpr int patch_member(int dx, int dy, int dz) {
  for (int k = 0; k < patch_Np<DIM, PATCH>(); ++k)
    if (patch_off<DIM, PATCH>(k, 0) == dx && patch_off<DIM, PATCH>(k, 1) == dy &&
        patch_off<DIM, PATCH>(k, 2) == dz)
      return k;
  return -1;
}

// Intergrid families (1D weights, Sec. 3.1): restriction r(t), prolongation p(t) = 2 r(t).
enum Family : int { FAM_LINEAR = 0, FAM_CUBIC = 1 };

__host__ __device__ constexpr int fam_radius(int fam) { return fam == FAM_LINEAR ? 1 : 2; }
// restriction weight at fine offset t from 2I (|t| <= radius)
__host__ __device__ constexpr double fam_r(int fam, int t) {
  return fam == FAM_LINEAR
             ? ((t == 0) ? 0.5 : ((t == 1 || t == -1) ? 0.25 : 0.0))
             : ((t == 0) ? 6.0 / 16 : ((t == 1 || t == -1) ? 4.0 / 16 : ((t == 2 || t == -2) ? 1.0 / 16 : 0.0)));
}
// 1D prolongation weight of coarse node J at fine node 2J + t
__host__ __device__ constexpr double fam_p(int fam, int t) { return 2.0 * fam_r(fam, t); }

// Weights of the compact 4th-order stencil, eq. (disc4thCompact) / (disc4thCompact3D), by
// the l1 distance of the offset from the centre: the Laplacian part L (times 1/h^2) and the
// mass part M.
template <int DIM>
__host__ __device__ constexpr double compact_L(int l1, double ih2) {
  // 2D: centre 10/3, axis -2/3, diagonal -1/6;  3D: centre 4, face -1/3, edge -1/6, corner 0
  return DIM == 2 ? (l1 == 0 ? 10.0 / 3 : l1 == 1 ? -2.0 / 3 : -1.0 / 6) * ih2
                  : (l1 == 0 ? 4.0 : l1 == 1 ? -1.0 / 3 : l1 == 2 ? -1.0 / 6 : 0.0) * ih2;
}
template <int DIM>
__host__ __device__ constexpr double compact_M(int l1) {
  // 2D: centre 2/3, axis 1/12;  3D: centre 1/2, axis 1/12
  return l1 == 0 ? (DIM == 2 ? 2.0 / 3 : 0.5) : (l1 == 1 ? 1.0 / 12 : 0.0);
}

// ---------------------------------------------------------------- launch helpers
// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD owns one
// contiguous range of the domain (its L2 then sees neighbouring rows).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, j = b >> 3, q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + j;
}

}  // namespace vh
