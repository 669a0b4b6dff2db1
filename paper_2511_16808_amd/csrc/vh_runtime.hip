// vh_runtime.hip -- host runtime and C ABI (include/vh.h) of the gfx950 solver.
//
// Owns the device hierarchy, drives the V-cycle (Sec. 2.2) and FGMRES(m)
// (Sec. 2.3).  Every arithmetic step runs in the kernels of vh_kernels.hip; the
// host only sequences launches and reads back one residual estimate per Arnoldi
// step to decide when to stop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vh.h"
#include "vh_internal.h"
#include "vh_launch.h"

using namespace vh;

namespace {

thread_local std::string g_last_error;

vh_status fail(vh_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

}  // namespace

// shared with the server translation unit
void vh_internal_set_error(const std::string& msg) { g_last_error = msg; }

namespace {

#define VH_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? VH_ENOMEM : VH_EDEVICE,                         \
                  std::string(#call) + ": " + hipGetErrorString(e_));                        \
  } while (0)

#define VH_TRY(expr)                \
  do {                              \
    vh_status s_ = (expr);          \
    if (s_ != VH_OK) return s_;     \
  } while (0)

constexpr int SM_SYMHALF = 6;
// warm-up iterations before the convergence factor of eq. (cf) is counted (Sec. 5.1)
constexpr int CF_WARMUP = 5;  // Level.form of the symmetric half of the assembled stencil

struct Level {
  Grid g{};
  int shape = CROSS;  // stencil shape of H_s^l
  int K = 0;
  void* A = nullptr;  // H_s^l, [K][N], preconditioner precision
  void* B = nullptr;  // smoother entries [E][N] (per-patch or assembled)
  int E = 0;
  void* q = nullptr;  // right-hand side, solution, residual (preconditioner precision)
  void* u = nullptr;
  void* r = nullptr;
  int rf = FAM_LINEAR, pf = FAM_LINEAR;  // transfers to level l+1
  double w = 1.0;                         // damping
  size_t bytes = 0;
  int patch = VH_PATCH_FULL;              // patch kind of this level's smoother
  int form = 0;                           // sweep form: the patch kind, 2 = assembled,
                                          // SM_SYMHALF = its symmetric half
  int mfma_txp[7] = {0, 0, 0, 0, 0, 0, 0};  // tuned matrix-core sweep tile per log2(S)
  int mfma_rows[7] = {0, 0, 0, 0, 0, 0, 0};
  int s64_tile = 0;   // variant of the 64-source 2D assembled sweep (0: not chosen yet)
  int s64_stile = 0;  // variant of the 64-source 2D stencil (operator, residual)
  // residual formed inside the sweep / the restriction (chosen per level at setup)
  bool fuse_sweep = false, fuse_restrict = false;
  bool nopiv = false;  // patch inverses eliminated without pivoting
  int sym_planes = -1;    // 3D symmetric half: planes per workgroup of the z walk (or -1)
  void* carry = nullptr;  // the walk's mirrored sums handed between chunks of planes
};

}  // namespace

struct vh_handle {
  int dim = 2;
  int n[3] = {1, 1, 1};
  double h = 0, omega = 0, shift = 0;
  int levels = 1;
  int patch = VH_PATCH_FULL;
  vh_options opt{};
  int prec = PREC_F64;
  size_t esz = 16;  // bytes per complex at the preconditioner precision
  hipStream_t s = nullptr;
  std::vector<Level> L;
  cpx<double>* Hfine = nullptr;  // unshifted finest operator, FP64 [K0][N]
  cpx<double>* Dinv = nullptr;   // inverse of the coarsest operator, FP64 dense
  int nc = 0;
  // FGMRES workspace
  int m = 20;
  cpx<double>* V = nullptr;  // (m+1) x N
  void* Z = nullptr;         // m x N at the preconditioner precision
  cpx<double>* part = nullptr;
  int nred = 512;   // blocks of the Krylov partial sums: enough waves to fill the GPU
  int bnred = 512;  // same for the multi-source path
  KrylovDev* K = nullptr;
  double* hstat = nullptr;  // pinned host copy of K->status
  // one-source FGMRES state for the delayed reorthogonalisation (source slot 0 of the
  // multi-source state, with its own partial-sum rows)
  BatchKrylovDev* dK = nullptr;
  cpx<double>* dpart = nullptr;
  int dnb = 512;
  // marks the copy of an Arnoldi step's status to the host, so that the host waits for
  // that copy while the step's update pass is already queued behind it
  hipEvent_t sev = nullptr;
  std::vector<void*> allocs;
  std::vector<size_t> alloc_sizes;
  // Region mode (a handle built inside memory handed over by the request server): every
  // allocation is carved out of [region, region + region_bytes) with no hipMalloc or
  // hipFree, the long-lived arrays from the bottom up and the set-up temporaries (FP64
  // Galerkin copies of a complex64 hierarchy, slab buffers, pivoting arrays) from the
  // top down, so the temporaries' space is reused by the solve workspace allocated after
  // them.  alloc_temp flags the top-down blocks; lo and hi are the two stack ends.
  char* region = nullptr;
  size_t region_bytes = 0, lo = 0, hi = 0;
  std::vector<char> alloc_temp, alloc_freed;
  double* pinned_ext = nullptr;  // server-owned pinned status buffer (4 + 256 doubles)
  size_t bytes = 0;       // device bytes held now
  size_t peak_bytes = 0;  // largest value bytes has taken
  double setup_ms = 0.0;  // wall time of vh_setup
  double moved = 0.0;     // algorithmic bytes of the kernels enqueued since the last reset
  // optional event timing (vh_options.timing): pairs of events with a kind tag
  // (0 = finest smoothing from u = 0, 1 = finest smoothing u += B r, 2 = V-cycle)
  // multi-source workspace, allocated on the first batched solve for up to bS sources
  int bS = 0;
  cpx<double>* bV = nullptr;  // (m+1) x N x bS
  void* bZ = nullptr;         // m x N x bS (preconditioner precision)
  cpx<double>* bQ = nullptr;  // right-hand sides, N x bS
  cpx<double>* bX = nullptr;  // iterates, N x bS
  cpx<double>* bpart = nullptr;
  BatchKrylovDev* bK = nullptr;
  double* bstat = nullptr;    // pinned, 64 x 4
  std::vector<void*> bq, bu, br;  // per-level V-cycle vectors, N_l x bS
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  int ev_used = 0;
  double t_ms[3] = {0, 0, 0};
  int t_n[3] = {0, 0, 0};

  ~vh_handle() {
    if (sev) (void)hipEventDestroy(sev);
    if (!region)
      for (void* p : allocs) (void)hipFree(p);
    if (!pinned_ext) {
      if (hstat) (void)hipHostFree(hstat);
      if (bstat) (void)hipHostFree(bstat);
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  // returns the index of a free event pair, or -1 if timing is off / the pool is full
  int tbegin(int kind) {
    if (!opt.timing || ev_used >= (int)ev_kind.size()) return -1;
    const int k = ev_used++;
    ev_kind[k] = kind;
    (void)hipEventRecord(ev[2 * k], s);
    return k;
  }
  void tend(int k) {
    if (k >= 0) (void)hipEventRecord(ev[2 * k + 1], s);
  }
  // call only after the stream has been synchronised
  void tflush() {
    for (int k = 0; k < ev_used; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess) {
        t_ms[ev_kind[k]] += ms;
        t_n[ev_kind[k]] += 1;
      }
    }
    ev_used = 0;
  }
  vh_status alloc(void** p, size_t bytes_, bool temp = false) {
    *p = nullptr;
    if (bytes_ == 0) return VH_OK;
    if (region) {
      const size_t a = (bytes_ + 255) / 256 * 256;
      if (a > hi - lo)
        return fail(VH_ENOMEM, "the request's device region is exhausted (" +
                                   std::to_string(bytes_) + " more bytes)");
      if (temp) {
        hi -= a;
        *p = region + hi;
      } else {
        *p = region + lo;
        lo += a;
      }
      bytes_ = a;
    } else {
      hipError_t e = hipMalloc(p, bytes_);
      if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(VH_ENOMEM, "hipMalloc of " + std::to_string(bytes_) + " bytes failed: " +
                                   hipGetErrorString(e));
      }
    }
    allocs.push_back(*p);
    alloc_sizes.push_back(bytes_);
    alloc_temp.push_back(temp ? 1 : 0);
    alloc_freed.push_back(0);
    bytes += bytes_;
    if (bytes > peak_bytes) peak_bytes = bytes;
    return VH_OK;
  }
  void release(void* p) {
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p && !alloc_freed[i]) {
        bytes -= alloc_sizes[i];
        if (!region) {
          (void)hipFree(p);
          allocs.erase(allocs.begin() + i);
          alloc_sizes.erase(alloc_sizes.begin() + i);
          alloc_temp.erase(alloc_temp.begin() + i);
          alloc_freed.erase(alloc_freed.begin() + i);
          return;
        }
        alloc_freed[i] = 1;
        // give back freed blocks at either stack end (a block freed out of order waits
        // until the blocks above it are freed)
        bool moved = true;
        while (moved) {
          moved = false;
          for (size_t k = 0; k < allocs.size(); ++k) {
            if (!alloc_freed[k] || alloc_freed[k] == 2) continue;
            const size_t off = (size_t)((char*)allocs[k] - region);
            if (alloc_temp[k] && off == hi) {
              hi += alloc_sizes[k];
              alloc_freed[k] = 2;
              moved = true;
            } else if (!alloc_temp[k] && off + alloc_sizes[k] == lo) {
              lo -= alloc_sizes[k];
              alloc_freed[k] = 2;
              moved = true;
            }
          }
        }
        return;
      }
  }
};

namespace {

int shape_points(int dim, int shape) {
  if (shape == CROSS) return 2 * dim + 1;
  int w = 2 * shape + 1;
  return dim == 2 ? w * w : w * w * w;
}

void shape_offsets(int dim, int shape, int K, int out[][3]) {
  for (int k = 0; k < K; ++k) {
    if (shape == CROSS) {
      out[k][0] = out[k][1] = out[k][2] = 0;
      if (k > 0) out[k][(k - 1) / 2] = ((k - 1) % 2 == 0) ? -1 : 1;
    } else {
      const int w = 2 * shape + 1;
      out[k][0] = k % w - shape;
      out[k][1] = (k / w) % w - shape;
      out[k][2] = dim == 3 ? k / (w * w) - shape : 0;
    }
  }
}

int patch_size(int dim, int patch) {
  switch (patch) {
    case VH_PATCH_FULL: return dim == 2 ? 9 : 27;
    case VH_PATCH_PLUS: return 2 * dim + 1;
    case VH_PATCH_RB: return dim == 2 ? 5 : 13;
    case VH_PATCH_ELEMENT: return dim == 2 ? 4 : 8;
    default: return 1;
  }
}

// damping used when the caller passes none.  Element, Plus, RB: Table "relaxParam"
// (2D columns; 3D columns for Element and Plus, the 3D RB patch, absent from the table,
// takes the Plus column).  Full patch: LFA smoothing-factor minimiser on the finest
// level and an exhaustive per-level search (not in the table; in 3D the search ran on
// the 257^3 geophysical medium with 6 levels, scored by FGMRES iterations).  Point patch (damped
// Jacobi): the table's Jacobi column with the compact stencil, for which the table was
// made; the LFA minimiser with the 2nd-order stencil.
double default_damping(int dim, int patch, int level, int stencil) {
  static const double jac2[] = {0.89, 0.9, 0.3, 0.71};
  static const double jac3[] = {0.6, 0.4, 0.3, 0.5};
  if (patch == VH_PATCH_POINT && stencil == VH_STENCIL_COMPACT4)
    return (dim == 2 ? jac2 : jac3)[level < 3 ? level : 3];
  static const double full2[] = {0.94, 1.2, 0.4, 0.6};
  static const double full3[] = {1.08, 0.5, 1.0, 0.4};
  static const double point2[] = {0.78, 0.7, 0.4, 0.6};
  static const double point3[] = {0.84, 0.7, 0.5, 0.5};
  static const double elem2[] = {0.97, 0.66, 0.48, 0.88};
  static const double plus2[] = {0.87, 0.57, 0.55, 0.74};
  static const double rb2[] = {0.83, 0.5, 0.4, 0.65};
  static const double elem3[] = {1.1, 0.7, 0.45, 0.6};
  static const double plus3[] = {0.92, 0.55, 0.45, 0.55};
  const double* t;
  switch (patch) {
    case VH_PATCH_FULL: t = dim == 2 ? full2 : full3; break;
    case VH_PATCH_ELEMENT: t = dim == 2 ? elem2 : elem3; break;
    case VH_PATCH_PLUS: t = dim == 2 ? plus2 : plus3; break;
    case VH_PATCH_RB: t = dim == 2 ? rb2 : plus3; break;
    default: t = dim == 2 ? point2 : point3;
  }
  return t[level < 3 ? level : 3];
}

vh_status validate(int dim, const int* n, double h, double omega, double shift, int levels,
                   int patch, const vh_options& o) {
  if (dim != 2 && dim != 3) return fail(VH_EINVAL, "dim must be 2 or 3");
  if (!n) return fail(VH_EINVAL, "n is NULL");
  if (!(h > 0) || !std::isfinite(h)) return fail(VH_EINVAL, "h must be positive");
  if (!(omega >= 0) || !std::isfinite(omega)) return fail(VH_EINVAL, "omega must be >= 0");
  if (!(shift >= 0) || !std::isfinite(shift)) return fail(VH_EINVAL, "shift must be >= 0");
  if (levels < 1 || levels > 16) return fail(VH_EINVAL, "levels must be in [1, 16]");
  if (patch != VH_PATCH_FULL && patch != VH_PATCH_POINT && patch != VH_PATCH_PLUS &&
      patch != VH_PATCH_RB && patch != VH_PATCH_ELEMENT)
    return fail(VH_EINVAL, "unknown patch");
  long long N = 1;
  for (int d = 0; d < dim; ++d) {
    if (n[d] < 3) return fail(VH_EINVAL, "every dimension needs >= 3 nodes");
    const long long c = n[d] - 1;
    const long long div = 1LL << (levels - 1);
    if (c % div != 0)
      return fail(VH_EINVAL, "(n[d]-1) must be divisible by 2^(levels-1)");
    if (c / div < 2) return fail(VH_EINVAL, "the coarsest level needs >= 3 nodes per dimension");
    N *= n[d];
  }
  if (N >= (1LL << 31)) return fail(VH_EINVAL, "grid too large (N >= 2^31)");
  if (o.precision != VH_PREC_FP64 && o.precision != VH_PREC_C64)
    return fail(VH_EINVAL, "unknown precision");
  if (o.restart < 1 || o.restart > MMAX) return fail(VH_EINVAL, "restart must be in [1, 64]");
  if (o.maxit < 1) return fail(VH_EINVAL, "maxit must be >= 1");
  if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 8 || o.nu2 > 8)
    return fail(VH_EINVAL, "nu1, nu2 must be in [0, 8] with nu1 + nu2 >= 1");
  if (o.bc != VH_BC_ABC && o.bc != VH_BC_DIRICHLET) return fail(VH_EINVAL, "unknown bc");
  if (o.stencil != VH_STENCIL_FD2 && o.stencil != VH_STENCIL_COMPACT4)
    return fail(VH_EINVAL, "unknown stencil");
  if (o.cycle != VH_CYCLE_V && o.cycle != VH_CYCLE_W) return fail(VH_EINVAL, "unknown cycle");
  if (o.fine_patch != -1 && o.fine_patch != VH_PATCH_FULL && o.fine_patch != VH_PATCH_POINT &&
      o.fine_patch != VH_PATCH_PLUS && o.fine_patch != VH_PATCH_RB &&
      o.fine_patch != VH_PATCH_ELEMENT)
    return fail(VH_EINVAL, "unknown fine_patch");
  if (o.smoother != VH_SMOOTHER_PATCH && o.smoother != VH_SMOOTHER_ASSEMBLED &&
      o.smoother != VH_SMOOTHER_SYMMETRIC)
    return fail(VH_EINVAL, "unknown smoother");
  if (o.smoother == VH_SMOOTHER_SYMMETRIC &&
      (patch != VH_PATCH_FULL || (o.fine_patch != -1 && o.fine_patch != VH_PATCH_FULL) ||
       o.stencil != VH_STENCIL_FD2 || o.batch != 0 || o.contraction != VH_CONTRACT_VALU))
    return fail(VH_EUNSUPPORTED,
                "the symmetric smoother needs the Full patch, the 5/7-point stencil, batch = 0 "
                "and the VALU contraction");
  if (o.ndamping < 0 || o.ndamping > 16) return fail(VH_EINVAL, "ndamping must be in [0, 16]");
  for (int k = 0; k < o.ndamping; ++k)
    if (!std::isfinite(o.damping[k])) return fail(VH_EINVAL, "damping values must be finite");
  if (o.smoother == VH_SMOOTHER_SYMMETRIC)
    for (int k = 0; k < o.ndamping; ++k)
      if (!(o.damping[k] > 0.0))
        return fail(VH_EINVAL, "the symmetric smoother needs damping > 0 on every level");
  if (o.contraction < VH_CONTRACT_VALU || o.contraction > VH_CONTRACT_MFMA_BF16X3)
    return fail(VH_EINVAL, "unknown contraction");
  if (o.sweep_tile < 0 || o.sweep_tile > S64_TILES)
    return fail(VH_EINVAL, "sweep_tile must be in [0, 10]");
  if (o.split_residual < 0 || o.split_residual > 2)
    return fail(VH_EINVAL, "split_residual must be 0, 1 or 2");
  if (o.sym_planes < -1 || o.sym_planes == 1 || o.sym_planes > 64)
    return fail(VH_EINVAL, "sym_planes must be -1, 0 or in [2, 64]");
  if (o.setup_pivot < 0 || o.setup_pivot > 1) return fail(VH_EINVAL, "setup_pivot must be 0 or 1");
  if (o.contraction != VH_CONTRACT_VALU &&
      (dim != 2 || patch != VH_PATCH_FULL || (o.fine_patch != -1 && o.fine_patch != VH_PATCH_FULL) ||
       o.smoother != VH_SMOOTHER_PATCH ||
       o.precision != VH_PREC_C64))
    return fail(VH_EUNSUPPORTED,
                "the matrix-core contraction needs dim 2, the Full patch, the per-patch "
                "smoother and the complex64 preconditioner");
  // the coarsest level is solved by a dense inverse
  long long nc = 1;
  for (int d = 0; d < dim; ++d) nc *= (n[d] - 1) / (1LL << (levels - 1)) + 1;
  if (nc > 8192) return fail(VH_EINVAL, "coarsest level too large for the dense solve (> 8192 nodes)");
  return VH_OK;
}

int resolve_intergrid(int dim, int ig) {
  if (ig < 0) return dim == 2 ? VH_IG_LEVDEP : VH_IG_LINEAR;
  return ig;
}

// (R family, P family, output shape) for the transfer from level l with shape `sin`
vh_status transfer_plan(int dim, int ig, int l, int sin, int* rf, int* pf, int* sout) {
  if (ig == VH_IG_LINEAR) {
    *rf = FAM_LINEAR;
    *pf = FAM_LINEAR;
    *sout = BOX1;
    return VH_OK;
  }
  if (dim == 3) return fail(VH_EUNSUPPORTED, "3D supports only the trilinear intergrid");
  if (ig == VH_IG_LEVDEP) {
    *rf = (l == 0) ? FAM_CUBIC : FAM_LINEAR;
    *pf = FAM_CUBIC;
    *sout = BOX2;
    return VH_OK;
  }
  if (ig == VH_IG_CUBIC) {  // R A P with radii 2 + r + 2 over 2: 5x5 from the finest, 7x7 below
    *rf = FAM_CUBIC;
    *pf = FAM_CUBIC;
    *sout = (sin == CROSS || sin == BOX1) ? BOX2 : BOX3;
    return VH_OK;
  }
  if (ig == VH_IG_MIXED) {
    *rf = FAM_LINEAR;
    *pf = FAM_CUBIC;
    *sout = BOX2;
    return VH_OK;
  }
  return fail(VH_EINVAL, "unknown intergrid");
}

size_t vec_bytes(const vh_handle* hd, const Level& Lv) { return (size_t)Lv.g.N * hd->esz; }

// Algorithmic bytes of the enqueued kernels (every array touched once per kernel),
// summed into hd->moved for vh_solve_stats.bytes_moved.  Coefficients read per node by an
// operator application: the 5/7-point finest operator reads only its centre entries.
double coef_reads(const Level& Lv) { return Lv.g.offrule ? 1.0 : (double)Lv.K; }
void count(vh_handle* hd, double nodes, double per_node) { hd->moved += nodes * per_node; }

// ---------------------------------------------------------------- V-cycle
vh_status smooth(vh_handle* hd, Level& Lv, const void* r, void* u, bool zero) {
  const int tk = (&Lv == &hd->L[0]) ? hd->tbegin(zero ? 0 : 1) : -1;
  const int form = Lv.form;
  count(hd, (double)Lv.g.N, (double)hd->esz * (Lv.E + (zero ? 2 : 3)));
  if (form == SM_SYMHALF)
    VH_HIP(vanka_sweep_sym(hd->dim, Lv.g, hd->prec, Lv.B, Lv.w, r, u, zero, hd->s,
                           Lv.sym_planes, Lv.carry));
  else
    VH_HIP(vanka_sweep(hd->dim, form, Lv.g, hd->prec, Lv.B, r, u, zero, hd->s));
  hd->tend(tk);
  return VH_OK;
}

vh_status residual(vh_handle* hd, Level& Lv, const void* q, const void* u, void* r) {
  count(hd, (double)Lv.g.N, (double)hd->esz * (coef_reads(Lv) + 3));
  VH_HIP(stencil(hd->dim, Lv.shape, Lv.g, OP_RESID, hd->prec, Lv.A, hd->prec, u, hd->prec, q, r,
                 hd->s));
  return VH_OK;
}

// one smoothing step u_out = u_in + B (q - A u_in) in one launch (u_out != u_in)
vh_status smooth_fused(vh_handle* hd, Level& Lv, const void* q, const void* u_in, void* u_out) {
  const int tk = (&Lv == &hd->L[0]) ? hd->tbegin(1) : -1;
  count(hd, (double)Lv.g.N, (double)hd->esz * (Lv.E + coef_reads(Lv) + 3));
  VH_HIP(vanka_sweep_fused(hd->dim, Lv.form, Lv.shape, Lv.g, hd->prec, Lv.B, Lv.w, Lv.A, q, u_in,
                           u_out, hd->s));
  hd->tend(tk);
  return VH_OK;
}

bool fuses_sweep(const vh_handle*, const Level& Lv) { return Lv.fuse_sweep; }
bool fuses_restrict(const vh_handle*, const Level& Lv) { return Lv.fuse_restrict; }

// Per level, whether the residual is formed inside the smoothing sweep and inside the
// restriction (vh_options.split_residual): 1 never, 2 wherever a kernel exists, 0 where
// the one launch is measured faster than the two it replaces.  The fused tile stage forms
// the residual on the tile's halo too, so on operators of many points or on small grids
// it can cost more than the stored residual saves; the timing (each form twice, one warm-up
// and eight timed launches each time, on the level's own arrays; the fused form must be 5 %
// ahead) settles it.  The choice depends only on the
// device, the level's grid, operator and smoother form and the precision, so it is kept for
// the process; both paths give the same bits.
std::mutex g_fuse_mu;
std::map<std::tuple<int, int, int, int, int>, int> g_fuse_cache;

vh_status tune_fuse(vh_handle* hd) {
  const int mode = hd->opt.split_residual;
  int dev = 0;
  VH_HIP(hipGetDevice(&dev));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  vh_status st = VH_OK;
  for (int l = 0; l + 1 < hd->levels && st == VH_OK; ++l) {
    Level& Lv = hd->L[l];
    Level& Lc = hd->L[l + 1];
    const bool cs = fused_sweep_ok(hd->dim, Lv.form, Lv.shape);
    const bool cr = fused_restrict_ok(hd->dim, Lv.rf, Lv.shape);
    Lv.fuse_sweep = Lv.fuse_restrict = false;
    if (mode == 1 || (!cs && !cr)) continue;
    if (mode == 2) {
      Lv.fuse_sweep = cs;
      Lv.fuse_restrict = cr;
      continue;
    }
    const auto key = std::make_tuple(dev, Lv.g.nx, Lv.g.ny, Lv.g.nz,
                                     hd->prec | Lv.shape << 2 | Lv.form << 5 | Lv.rf << 9);
    {
      std::lock_guard<std::mutex> lock(g_fuse_mu);
      auto it = g_fuse_cache.find(key);
      if (it != g_fuse_cache.end()) {
        Lv.fuse_sweep = (it->second & 1) != 0;
        Lv.fuse_restrict = (it->second & 2) != 0;
        continue;
      }
    }
    if (!e0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
      st = fail(VH_EDEVICE, "hipEventCreate failed");
      break;
    }
    // the level's arrays hold zeros here (set-up has not run a cycle yet)
    auto split_sweep = [&]() {
      hipError_t e = stencil(hd->dim, Lv.shape, Lv.g, OP_RESID, hd->prec, Lv.A, hd->prec, Lv.u,
                             hd->prec, Lv.q, Lv.r, hd->s);
      if (e != hipSuccess) return e;
      return Lv.form == SM_SYMHALF
                 ? vanka_sweep_sym(hd->dim, Lv.g, hd->prec, Lv.B, Lv.w, Lv.r, Lv.u, false, hd->s,
                                   Lv.sym_planes, Lv.carry)
                 : vanka_sweep(hd->dim, Lv.form, Lv.g, hd->prec, Lv.B, Lv.r, Lv.u, false, hd->s);
    };
    auto fused_sweep = [&]() {
      return vanka_sweep_fused(hd->dim, Lv.form, Lv.shape, Lv.g, hd->prec, Lv.B, Lv.w, Lv.A,
                               Lv.q, Lv.u, Lv.r, hd->s);
    };
    auto split_restrict = [&]() {
      hipError_t e = stencil(hd->dim, Lv.shape, Lv.g, OP_RESID, hd->prec, Lv.A, hd->prec, Lv.u,
                             hd->prec, Lv.q, Lv.r, hd->s);
      if (e != hipSuccess) return e;
      return restrict_(hd->dim, Lv.rf, Lv.g, Lc.g, hd->prec, Lv.r, Lc.q, hd->s);
    };
    auto fused_restrict = [&]() {
      return resid_restrict(hd->dim, Lv.rf, Lv.shape, Lv.g, Lc.g, hd->prec, Lv.A, Lv.q, Lv.u,
                            Lc.q, hd->s);
    };
    auto timed = [&](auto&& f, float& ms) {
      float t = 0.f;
      hipError_t e = f();
      if (e == hipSuccess) e = hipEventRecord(e0, hd->s);
      for (int k = 0; k < 8 && e == hipSuccess; ++k) e = f();
      if (e == hipSuccess) e = hipEventRecord(e1, hd->s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      ms += t;
      return e;
    };
    // the two forms alternate twice; the fused one is taken only when it is clearly ahead
    auto pick = [&](auto&& split_f, auto&& fused_f, hipError_t& e) {
      float a = 0.f, b = 0.f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = timed(split_f, a);
        if (e == hipSuccess) e = timed(fused_f, b);
      }
      return e == hipSuccess && b < 0.95f * a;
    };
    hipError_t e = hipSuccess;
    if (cs) Lv.fuse_sweep = pick(split_sweep, fused_sweep, e);
    if (cr && e == hipSuccess) Lv.fuse_restrict = pick(split_restrict, fused_restrict, e);
    if (e != hipSuccess) {
      st = fail(VH_EDEVICE, std::string("fusion timing: ") + hipGetErrorString(e));
      break;
    }
    std::lock_guard<std::mutex> lock(g_fuse_mu);
    g_fuse_cache[key] = (Lv.fuse_sweep ? 1 : 0) | (Lv.fuse_restrict ? 2 : 0);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

// number of visits of level l + 1 from level l: two for a W-cycle unless l + 1 is the
// coarsest level (solved directly)
int coarse_visits(const vh_handle* hd, int l) {
  return (hd->opt.cycle == VH_CYCLE_W && l + 2 < hd->levels) ? 2 : 1;
}

// u <- cycle(l, q, u); u is taken as zero on entry when from_zero (its content is ignored).
// Where the level forms the residual inside its sweep, each such step writes a second
// array (the level's residual array, unused then); the first step of a run is placed so
// that the last one lands in u.
vh_status vcycle(vh_handle* hd, int l, const void* q, void* u, bool from_zero) {
  Level& Lv = hd->L[l];
  if (l == hd->levels - 1) {
    count(hd, (double)hd->nc, 16.0 * hd->nc + 2.0 * hd->esz);
    VH_HIP(dense_matvec(hd->nc, hd->Dinv, hd->prec, q, u, hd->s));
    return VH_OK;
  }
  const int nu1 = hd->opt.nu1, nu2 = hd->opt.nu2;
  const bool fs = fuses_sweep(hd, Lv);
  void* alt = Lv.r;
  if (nu1 == 0 && from_zero) {
    count(hd, (double)Lv.g.N, (double)hd->esz);
    VH_HIP(fill(u, (size_t)Lv.g.N, hd->prec, 0.0, 0.0, hd->s));
  }
  {
    int k = 0;
    void* cur = u;
    if (nu1 > 0 && from_zero) {  // u = 0: the first step is u = B q
      cur = (fs && (nu1 - 1) % 2 == 1) ? alt : u;
      VH_TRY(smooth(hd, Lv, q, cur, true));
      k = 1;
    }
    if (fs && cur == u && (nu1 - k) % 2 == 1) {  // an odd run from u: one step in place
      VH_TRY(residual(hd, Lv, q, u, Lv.r));
      VH_TRY(smooth(hd, Lv, Lv.r, u, false));
      ++k;
    }
    for (; k < nu1; ++k) {
      if (fs) {
        void* nxt = (cur == u) ? alt : u;
        VH_TRY(smooth_fused(hd, Lv, q, cur, nxt));
        cur = nxt;
      } else {
        VH_TRY(residual(hd, Lv, q, u, Lv.r));
        VH_TRY(smooth(hd, Lv, Lv.r, u, false));
      }
    }
  }
  Level& Lc = hd->L[l + 1];
  if (fuses_restrict(hd, Lv)) {
    count(hd, (double)Lv.g.N, (double)hd->esz * (coef_reads(Lv) + 2));
    count(hd, (double)Lc.g.N, (double)hd->esz);
    VH_HIP(resid_restrict(hd->dim, Lv.rf, Lv.shape, Lv.g, Lc.g, hd->prec, Lv.A, q, u, Lc.q,
                          hd->s));
  } else {
    VH_TRY(residual(hd, Lv, q, u, Lv.r));
    count(hd, (double)(Lv.g.N + Lc.g.N), (double)hd->esz);
    VH_HIP(restrict_(hd->dim, Lv.rf, Lv.g, Lc.g, hd->prec, Lv.r, Lc.q, hd->s));
  }
  for (int v = 0; v < coarse_visits(hd, l); ++v) VH_TRY(vcycle(hd, l + 1, Lc.q, Lc.u, v == 0));
  // the correction goes to the array the post-smoothing run starts from
  void* cur = (fs && nu2 % 2 == 1) ? alt : u;
  count(hd, (double)(2 * Lv.g.N + Lc.g.N), (double)hd->esz);
  VH_HIP(prolong_add(hd->dim, Lv.pf, Lv.g, Lc.g, hd->prec, Lc.u, cur, hd->s, u));
  for (int k = 0; k < nu2; ++k) {
    if (fs) {
      void* nxt = (cur == u) ? alt : u;
      VH_TRY(smooth_fused(hd, Lv, q, cur, nxt));
      cur = nxt;
    } else {
      VH_TRY(residual(hd, Lv, q, u, Lv.r));
      VH_TRY(smooth(hd, Lv, Lv.r, u, false));
    }
  }
  return VH_OK;
}

// z (preconditioner precision) = M^{-1} v (FP64)
vh_status precondition(vh_handle* hd, const cpx<double>* v, void* z) {
  Level& L0 = hd->L[0];
  const void* q = v;
  if (hd->prec != PREC_F64) {
    count(hd, (double)L0.g.N, 16.0 + hd->esz);
    VH_HIP(convert(v, PREC_F64, L0.q, hd->prec, (size_t)L0.g.N, hd->s));
    q = L0.q;
  }
  const int tk = hd->tbegin(2);
  VH_TRY(vcycle(hd, 0, q, z, true));
  hd->tend(tk);
  return VH_OK;
}

vh_status read_status(vh_handle* hd) {
  VH_HIP(hipMemcpyAsync(hd->hstat, hd->K->status, 4 * sizeof(double), hipMemcpyDeviceToHost,
                        hd->s));
  VH_HIP(hipStreamSynchronize(hd->s));
  hd->tflush();
  return VH_OK;
}

// ---------------------------------------------------------------- FGMRES(m)
// One source.  Arnoldi by classical Gram-Schmidt with one reorthogonalisation, delayed
// into the next step (one reduction pass and one update pass over the basis per step,
// the multi-source kernels on one source slot): step j applies the preconditioner to
// the lagged vector V_j and completes Hessenberg column j-1, so the residual estimate
// of an iteration is known one step later; a cycle that runs to m closes column m-1
// with one more reduction pass.
vh_status read_dstatus(vh_handle* hd) {
  VH_HIP(hipMemcpyAsync(hd->hstat, hd->dK->status, 4 * sizeof(double), hipMemcpyDeviceToHost,
                        hd->s));
  VH_HIP(hipStreamSynchronize(hd->s));
  hd->tflush();
  return VH_OK;
}

// the status copy of an Arnoldi step, marked by hd->sev; the host waits on the mark
// (status_wait) after it has queued the step's update pass, so the device is not idle
// while the host decides whether the cycle goes on (the pass is harmless if it stops:
// it touches neither the Hessenberg columns in use nor Z)
vh_status status_post(vh_handle* hd, const double* src, size_t bytes, double* dst) {
  VH_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, hd->s));
  VH_HIP(hipEventRecord(hd->sev, hd->s));
  return VH_OK;
}
vh_status status_wait(vh_handle* hd) {
  VH_HIP(hipEventSynchronize(hd->sev));
  hd->tflush();  // every timing event was recorded before the mark
  return VH_OK;
}

vh_status fgmres_one(vh_handle* hd, const cpx<double>* q, cpx<double>* x, double tol,
                     vh_solve_stats* st) {
  const size_t N = (size_t)hd->L[0].g.N;
  const int m = hd->m;
  BatchKrylovDev* K = hd->dK;
  cpx<double>* V = hd->V;
  auto Vj = [&](int j) { return V + (size_t)j * N; };
  auto Zj = [&](int j) { return (void*)((char*)hd->Z + (size_t)j * N * hd->esz); };
  const long long NL = (long long)N;

  const double dN = (double)N, k0 = coef_reads(hd->L[0]);
  count(hd, dN, 16.0);
  VH_HIP(fill(x, N, PREC_F64, 0.0, 0.0, hd->s));
  // r = q (x = 0); beta = ||q||; V_0 = r / beta
  auto restart_vector = [&]() -> vh_status {
    count(hd, dN, 48.0);  // norm pass and scaling of V_0
    VH_HIP(batch_cgs(2, V, N, 0, K->h2, Vj(0), NL, 0, hd->dpart, hd->dnb, K->nrm2, hd->s));
    VH_HIP(batch_cycle_init(K, m, 1, hd->s));
    VH_HIP(batch_scale(K, Vj(0), Vj(0), NL, 0, hd->s));
    return read_dstatus(hd);
  };
  count(hd, dN, 32.0);
  VH_HIP(hipMemcpyAsync(Vj(0), q, N * sizeof(cpx<double>), hipMemcpyDeviceToDevice, hd->s));
  VH_TRY(restart_vector());
  const double bnorm = hd->hstat[3];
  double beta = bnorm;
  int its = 0, restarts = 0;
  bool converged = false;
  double est = 1.0, est_w = NAN;  // residual estimate now and after CF_WARMUP iterations
  if (!(bnorm == bnorm) || std::isinf(bnorm)) return fail(VH_EBREAKDOWN, "non-finite right-hand side");
  if (bnorm == 0.0) {
    if (st) {
      *st = vh_solve_stats{};
      st->converged = 1;
      st->c_f = NAN;
    }
    return VH_OK;
  }
  while (true) {
    if (beta / bnorm <= tol) {
      converged = true;
      break;
    }
    if (its >= hd->opt.maxit) break;
    int k = 0;
    bool stop = false;
    // iteration `done` completed: read its estimate; true when the cycle ends here
    auto account = [&](int done, bool posted) -> vh_status {
      VH_TRY(posted ? status_wait(hd) : read_dstatus(hd));
      if (hd->hstat[2] != 0.0) return fail(VH_EBREAKDOWN, "NaN/Inf in the Arnoldi process");
      ++its;
      k = done;
      est = hd->hstat[0] / bnorm;
      if (its == CF_WARMUP) est_w = est;
      stop = est <= tol || its >= hd->opt.maxit || hd->hstat[1] == 0.0;
      return VH_OK;
    };
    // complex64 preconditioner: pass B leaves the next input already rounded in L0.q
    cpx<float>* lo = hd->prec == PREC_F32 ? (cpx<float>*)hd->L[0].q : nullptr;
    for (int j = 0; j < m && !stop; ++j) {
      if (j > 0 && lo) {
        const int tk = hd->tbegin(2);
        VH_TRY(vcycle(hd, 0, hd->L[0].q, Zj(j), true));
        hd->tend(tk);
      } else {
        VH_TRY(precondition(hd, Vj(j), Zj(j)));
      }
      count(hd, dN, 16.0 * k0 + hd->esz + 16.0);
      VH_HIP(stencil(hd->dim, hd->L[0].shape, hd->L[0].g, OP_APPLY, PREC_F64, hd->Hfine, hd->prec,
                     Zj(j), PREC_F64, nullptr, Vj(j + 1), hd->s));
      count(hd, dN, 16.0 * (2 * j + 6) + (lo ? 8.0 : 0.0));  // passes A and B
      VH_HIP(batch_dcgs_a(V, N, j, j + 1, NL, 0, hd->dpart, hd->dnb, K, hd->s));
      VH_HIP(batch_dcgs_fin(K, j, 1, 0, hd->s));
      if (j >= 1) VH_TRY(status_post(hd, K->status, 4 * sizeof(double), hd->hstat));
      VH_HIP(batch_dcgs_b(V, N, j, NL, 0, K, lo, hd->s));
      if (j >= 1) {
        VH_TRY(account(j, true));
        if (stop) break;
      }
    }
    if (!stop) {
      count(hd, dN, 16.0 * (m + 2));
      VH_HIP(batch_dcgs_a(V, N, m, m, NL, 0, hd->dpart, hd->dnb, K, hd->s));
      VH_HIP(batch_dcgs_fin(K, m, 1, 1, hd->s));
      VH_TRY(account(m, false));
    }
    VH_HIP(hipMemcpyAsync(K->kcols, &k, sizeof(int), hipMemcpyHostToDevice, hd->s));
    VH_HIP(batch_backsolve(K, 1, hd->s));
    count(hd, dN, (double)k * hd->esz + 32.0);
    VH_HIP(batch_update_x(K, k, hd->prec, hd->Z, N, x, NL, 0, hd->s));
    // true residual r = q - H x (FP64), V_0 = r / ||r||
    count(hd, dN, 16.0 * k0 + 48.0);
    VH_HIP(stencil(hd->dim, hd->L[0].shape, hd->L[0].g, OP_RESID, PREC_F64, hd->Hfine, PREC_F64, x,
                   PREC_F64, q, Vj(0), hd->s));
    VH_TRY(restart_vector());
    beta = hd->hstat[3];
    ++restarts;
    if (!(beta == beta) || std::isinf(beta)) return fail(VH_EBREAKDOWN, "non-finite residual");
  }
  if (st) {
    st->iterations = its;
    st->restarts = restarts;
    st->converged = converged ? 1 : 0;
    st->relres = beta / bnorm;
    st->relres_est = est;
    st->c_f = its > CF_WARMUP && est_w > 0.0 ? std::pow(est / est_w, 1.0 / (its - CF_WARMUP)) : NAN;
  }
  return converged ? VH_OK : fail(VH_ENOCONV, "maxit reached before tol");
}

// ---------------------------------------------------------------- multi-source path
vh_status ensure_batch(vh_handle* hd, int S) {
  if (hd->opt.smoother == VH_SMOOTHER_SYMMETRIC)
    return fail(VH_EUNSUPPORTED, "the multi-source sweeps do not take the symmetric smoother");
  if (hd->bS >= S) return VH_OK;
  // (re)allocate for S sources
  auto drop = [&](void* p) {
    if (p) {
      hd->release(p);
    }
  };
  drop(hd->bV);
  drop(hd->bZ);
  drop(hd->bQ);
  drop(hd->bX);
  drop(hd->bpart);
  drop(hd->bK);
  for (void* p : hd->bq) drop(p);
  for (void* p : hd->bu) drop(p);
  for (void* p : hd->br) drop(p);
  hd->bq.assign(hd->levels, nullptr);
  hd->bu.assign(hd->levels, nullptr);
  hd->br.assign(hd->levels, nullptr);
  hd->bS = 0;
  const size_t N = (size_t)hd->L[0].g.N;
  VH_TRY(hd->alloc((void**)&hd->bV, (size_t)(hd->m + 1) * N * S * sizeof(cpx<double>)));
  VH_TRY(hd->alloc(&hd->bZ, (size_t)hd->m * N * S * hd->esz));
  VH_TRY(hd->alloc((void**)&hd->bQ, N * S * sizeof(cpx<double>)));
  VH_TRY(hd->alloc((void**)&hd->bX, N * S * sizeof(cpx<double>)));
  {
    long long nb = (long long)N * S / 8192;
    hd->bnred = (int)(nb < 64 ? 64 : (nb > 1024 ? 1024 : nb));
  }
  // bnred partial rows of 65 x 64 sums, then 65 x 16 x 64 slice sums
  VH_TRY(hd->alloc((void**)&hd->bpart,
                   ((size_t)hd->bnred + 16) * 65 * 64 * sizeof(cpx<double>)));
  VH_TRY(hd->alloc((void**)&hd->bK, sizeof(BatchKrylovDev)));
  VH_HIP(hipMemsetAsync(hd->bK, 0, sizeof(BatchKrylovDev), hd->s));
  for (int l = 0; l < hd->levels; ++l) {
    const size_t Nl = (size_t)hd->L[l].g.N * S;
    VH_TRY(hd->alloc(&hd->bq[l], Nl * hd->esz));
    VH_TRY(hd->alloc(&hd->bu[l], Nl * hd->esz));
    VH_TRY(hd->alloc(&hd->br[l], Nl * hd->esz));
  }
  if (!hd->bstat && hd->pinned_ext) hd->bstat = hd->pinned_ext + 4;
  if (!hd->bstat) VH_HIP(hipHostMalloc((void**)&hd->bstat, 64 * 4 * sizeof(double), hipHostMallocDefault));
  hd->bS = S;
  return VH_OK;
}

vh_status bsmooth(vh_handle* hd, int l, int ls, const void* r, void* u, bool zero) {
  Level& Lv = hd->L[l];
  const int tk = (l == 0) ? hd->tbegin(zero ? 0 : 1) : -1;
  const int form = Lv.form;
  count(hd, (double)Lv.g.N, (double)hd->esz * (Lv.E + (zero ? 2 : 3) * (1 << ls)));
  if (Lv.mfma_txp[ls])
    VH_HIP(batch_sweep_mfma(Lv.g, ls, hd->opt.contraction == VH_CONTRACT_MFMA_BF16X3,
                            Lv.mfma_txp[ls], Lv.mfma_rows[ls], Lv.B, r, u, zero, hd->s));
  else
    VH_HIP(batch_sweep(hd->dim, form, Lv.g, ls, hd->prec, Lv.B, r, u, zero, hd->s, Lv.s64_tile));
  hd->tend(tk);
  return VH_OK;
}

// Tile choice of the matrix-core sweep for every smoothed level and batch width S:
// each candidate (patches per strip row, about 1, 2 or 4 blocks per CU) is timed on the
// level's own grid with HIP events, the fastest kept.  Runs once per handle and S, so
// repeated solves with one handle take the same tiles (and give the same bits).
vh_status tune_mfma(vh_handle* hd, int ls) {
  const int S = 1 << ls;
  if (hd->opt.contraction == VH_CONTRACT_VALU || ls < 4) return VH_OK;
  int dev = 0, ncu = 256;
  VH_HIP(hipGetDevice(&dev));
  VH_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int split = hd->opt.contraction == VH_CONTRACT_MFMA_BF16X3;
  hipEvent_t e0, e1;
  VH_HIP(hipEventCreate(&e0));
  VH_HIP(hipEventCreate(&e1));
  vh_status st = VH_OK;
  for (int l = 0; l + 1 < hd->levels && st == VH_OK; ++l) {
    Level& Lv = hd->L[l];
    if (Lv.mfma_txp[ls]) continue;
    const size_t NS = (size_t)Lv.g.N * S;
    if (fill(hd->br[l], NS, hd->prec, 0, 0, hd->s) != hipSuccess) { st = VH_EDEVICE; break; }
    float best = 1e30f;
    int btxp = 16, brows = Lv.g.ny;
    for (int txp : {16, 32}) {
      const long long nstrip = (Lv.g.nx + txp - 3) / (txp - 2);
      for (int per_cu : {1, 2, 4}) {
        long long nchunk = (long long)per_cu * ncu / nstrip;
        if (nchunk < 1) nchunk = 1;
        if (nchunk > Lv.g.ny) nchunk = Lv.g.ny;
        const int rows = (int)((Lv.g.ny + nchunk - 1) / nchunk);
        float ms = 0.f;
        hipError_t e = batch_sweep_mfma(Lv.g, ls, split, txp, rows, Lv.B, hd->br[l], hd->bu[l],
                                        true, hd->s);
        if (e == hipSuccess) e = hipEventRecord(e0, hd->s);
        for (int k = 0; k < 3 && e == hipSuccess; ++k)
          e = batch_sweep_mfma(Lv.g, ls, split, txp, rows, Lv.B, hd->br[l], hd->bu[l], true,
                               hd->s);
        if (e == hipSuccess) e = hipEventRecord(e1, hd->s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          continue;  // a tile that does not launch here is not a candidate
        }
        if (ms < best) {
          best = ms;
          btxp = txp;
          brows = rows;
        }
      }
    }
    if (best >= 1e30f) {
      st = fail(VH_EDEVICE, "no matrix-core sweep tile launches on this device");
      break;
    }
    Lv.mfma_txp[ls] = btxp;
    Lv.mfma_rows[ls] = brows;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Variants of the 64-source 2D assembled sweep and of the 64-source 2D stencil (residual,
// operator) for every smoothed level: the caller's vh_options.sweep_tile, else the fastest
// of the S64_TILES candidates of each, timed with HIP events on the level's own grid (one
// warm-up and three timed launches each).  The
// choice depends only on the device, the grid and the precision, so it is kept for the
// process and reused by later handles; every candidate computes the same sums in the same
// order, so the choice does not change any result bit.
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int, int>, int> g_tile_cache;

vh_status tune_s64(vh_handle* hd, int ls) {
  if (ls != 6 || hd->dim != 2 || hd->opt.contraction != VH_CONTRACT_VALU) return VH_OK;
  int dev = 0;
  VH_HIP(hipGetDevice(&dev));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  vh_status st = VH_OK;
  for (int l = 0; l + 1 < hd->levels && st == VH_OK; ++l) {
    Level& Lv = hd->L[l];
    if (Lv.s64_tile) continue;
    if (hd->opt.sweep_tile > 0) {
      Lv.s64_tile = Lv.s64_stile = hd->opt.sweep_tile;
      continue;
    }
    const auto key = std::make_tuple(dev, Lv.g.nx, Lv.g.ny, hd->prec * 16 + Lv.shape * 4 + Lv.form);
    {
      std::lock_guard<std::mutex> lock(g_tile_mu);
      auto it = g_tile_cache.find(key);
      if (it != g_tile_cache.end()) {
        Lv.s64_tile = it->second & 0xff;
        Lv.s64_stile = it->second >> 8;
        continue;
      }
    }
    if (!e0) {
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(VH_EDEVICE, "hipEventCreate failed");
        break;
      }
    }
    const size_t NS = (size_t)Lv.g.N << ls;
    if (fill(hd->br[l], NS, hd->prec, 0, 0, hd->s) != hipSuccess ||
        fill(hd->bu[l], NS, hd->prec, 0, 0, hd->s) != hipSuccess) {
      st = fail(VH_EDEVICE, "fill failed");
      break;
    }
    // which = 0: the sweep (assembled form only), 1: the residual with the level operator
    int chosen[2] = {S64_DEFAULT_TILE, S64_DEFAULT_TILE};
    for (int which = 0; which < 2 && st == VH_OK; ++which) {
      if (which == 0 && Lv.form != 2) continue;
      auto launch = [&](int t) {
        return which == 0 ? batch_sweep(2, 2, Lv.g, ls, hd->prec, Lv.B, hd->br[l], hd->bu[l],
                                        false, hd->s, t)
                          : batch_stencil(2, Lv.shape, Lv.g, ls, OP_RESID, hd->prec, Lv.A,
                                          hd->prec, hd->bu[l], hd->prec, hd->bu[l], hd->br[l],
                                          hd->s, t);
      };
      float best = 1e30f;
      for (int t = 1; t <= S64_TILES; ++t) {
        float ms = 0.f;
        hipError_t e = launch(t);
        if (e == hipSuccess) e = hipEventRecord(e0, hd->s);
        for (int k = 0; k < 3 && e == hipSuccess; ++k) e = launch(t);
        if (e == hipSuccess) e = hipEventRecord(e1, hd->s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = fail(VH_EDEVICE, std::string("tile timing: ") + hipGetErrorString(e));
          break;
        }
        if (ms < best) {
          best = ms;
          chosen[which] = t;
        }
      }
    }
    if (st != VH_OK) break;
    Lv.s64_tile = chosen[0];
    Lv.s64_stile = chosen[1];
    std::lock_guard<std::mutex> lock(g_tile_mu);
    g_tile_cache[key] = chosen[0] | (chosen[1] << 8);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

vh_status bresidual(vh_handle* hd, int l, int ls, const void* q, const void* u, void* r) {
  Level& Lv = hd->L[l];
  count(hd, (double)Lv.g.N, (double)hd->esz * (coef_reads(Lv) + 3 * (1 << ls)));
  VH_HIP(batch_stencil(hd->dim, Lv.shape, Lv.g, ls, OP_RESID, hd->prec, Lv.A, hd->prec, u,
                       hd->prec, q, r, hd->s, Lv.s64_stile));
  return VH_OK;
}

// the V-cycle of vcycle() on a batch of 1 << ls sources
vh_status vcycle_b(vh_handle* hd, int l, int ls, const void* q, void* u, bool from_zero) {
  Level& Lv = hd->L[l];
  const double S = (double)(1 << ls);
  if (l == hd->levels - 1) {
    count(hd, (double)hd->nc, 16.0 * hd->nc + 2.0 * S * hd->esz);
    VH_HIP(batch_dense(hd->nc, ls, hd->Dinv, hd->prec, q, u, hd->s));
    return VH_OK;
  }
  const int nu1 = hd->opt.nu1, nu2 = hd->opt.nu2;
  void* r = hd->br[l];
  if (nu1 == 0 && from_zero) {
    count(hd, (double)Lv.g.N, S * hd->esz);
    VH_HIP(fill(u, (size_t)Lv.g.N << ls, hd->prec, 0.0, 0.0, hd->s));
  }
  for (int k = 0; k < nu1; ++k) {
    if (k == 0 && from_zero) {
      VH_TRY(bsmooth(hd, l, ls, q, u, true));
    } else {
      VH_TRY(bresidual(hd, l, ls, q, u, r));
      VH_TRY(bsmooth(hd, l, ls, r, u, false));
    }
  }
  Level& Lc = hd->L[l + 1];
  VH_TRY(bresidual(hd, l, ls, q, u, r));
  count(hd, (double)(Lv.g.N + Lc.g.N), S * hd->esz);
  VH_HIP(batch_restrict(hd->dim, Lv.rf, Lv.g, Lc.g, ls, hd->prec, r, hd->bq[l + 1], hd->s));
  for (int v = 0; v < coarse_visits(hd, l); ++v)
    VH_TRY(vcycle_b(hd, l + 1, ls, hd->bq[l + 1], hd->bu[l + 1], v == 0));
  count(hd, (double)(2 * Lv.g.N + Lc.g.N), S * hd->esz);
  VH_HIP(batch_prolong_add(hd->dim, Lv.pf, Lv.g, Lc.g, ls, hd->prec, hd->bu[l + 1], u, hd->s));
  for (int k = 0; k < nu2; ++k) {
    VH_TRY(bresidual(hd, l, ls, q, u, r));
    VH_TRY(bsmooth(hd, l, ls, r, u, false));
  }
  return VH_OK;
}

vh_status read_bstatus(vh_handle* hd, int S) {
  VH_HIP(hipMemcpyAsync(hd->bstat, hd->bK->status, (size_t)S * 4 * sizeof(double),
                        hipMemcpyDeviceToHost, hd->s));
  VH_HIP(hipStreamSynchronize(hd->s));
  hd->tflush();
  return VH_OK;
}

// FGMRES(m) for nsrc <= 64 sources sharing every V-cycle.  The sources advance in
// lockstep; a source that reaches tol (or maxit) inside a cycle freezes: its solution
// update uses only its own columns and it takes no further updates.
vh_status fgmres_batch(vh_handle* hd, const cpx<double>* q, int nsrc, cpx<double>* u, double tol,
                       vh_solve_stats* st) {
  int ls = 0;
  while ((1 << ls) < nsrc) ++ls;
  const int S = 1 << ls;
  VH_TRY(ensure_batch(hd, S));
  VH_TRY(tune_mfma(hd, ls));
  VH_TRY(tune_s64(hd, ls));
  const long long N = hd->L[0].g.N;
  const int m = hd->m;
  const size_t ldv = (size_t)N * S;
  BatchKrylovDev* K = hd->bK;
  auto Vj = [&](int j) { return hd->bV + (size_t)j * ldv; };
  auto Zj = [&](int j) { return (void*)((char*)hd->bZ + (size_t)j * ldv * hd->esz); };
  const Grid g0 = hd->L[0].g;
  hipStream_t s = hd->s;

  const double dNS = (double)N * S, k0 = coef_reads(hd->L[0]);
  count(hd, dNS, 32.0 + 16.0 + 32.0 + 48.0);  // gather, zero x, copy to V_0, norm and scale
  VH_HIP(batch_gather(N, S, nsrc, q, hd->bQ, s));
  VH_HIP(fill(hd->bX, (size_t)N * S, PREC_F64, 0, 0, s));
  VH_HIP(hipMemcpyAsync(Vj(0), hd->bQ, ldv * sizeof(cpx<double>), hipMemcpyDeviceToDevice, s));
  VH_HIP(batch_cgs(2, hd->bV, ldv, 0, K->h2, Vj(0), N, ls, hd->bpart, hd->bnred, K->nrm2, s));
  VH_HIP(batch_cycle_init(K, m, S, s));
  VH_HIP(batch_scale(K, Vj(0), Vj(0), N, ls, s));
  VH_TRY(read_bstatus(hd, S));
  std::vector<double> bnorm(S), beta(S);
  std::vector<int> its(S, 0), restarts(S, 0), active(S, 0), conv(S, 0);
  std::vector<double> est(S, 1.0), est_w(S, NAN);
  for (int k = 0; k < S; ++k) {
    bnorm[k] = hd->bstat[k * 4 + 3];
    beta[k] = bnorm[k];
    if (k < nsrc && !(bnorm[k] == bnorm[k] && !std::isinf(bnorm[k])))
      return fail(VH_EBREAKDOWN, "non-finite right-hand side");
    if (k < nsrc && bnorm[k] > 0) active[k] = 1;
    if (k < nsrc && bnorm[k] == 0) conv[k] = 1;
  }
  int kcols[64];
  while (true) {
    bool any = false;
    for (int k = 0; k < S; ++k) {
      if (!active[k]) continue;
      if (beta[k] / bnorm[k] <= tol) {
        active[k] = 0;
        conv[k] = 1;
      } else if (its[k] >= hd->opt.maxit) {
        active[k] = 0;
      }
      any = any || active[k];
    }
    if (!any) break;
    std::vector<int> stopped(S, 0);
    for (int k = 0; k < S; ++k) kcols[k] = 0;
    // Arnoldi with delayed reorthogonalisation: step j applies the preconditioner to the
    // lagged vector V_j and completes Hessenberg column j-1 (iteration j), so the
    // residual estimate of an iteration is known one step later; a cycle that runs to m
    // closes column m-1 with one more reduction pass.
    auto account = [&](int done, bool posted) -> vh_status {
      VH_TRY(posted ? status_wait(hd) : read_bstatus(hd, S));
      bool all_stopped = true;
      for (int k = 0; k < S; ++k) {
        if (!active[k] || stopped[k]) continue;
        if (hd->bstat[k * 4 + 2] != 0.0) return fail(VH_EBREAKDOWN, "NaN/Inf in the Arnoldi process");
        ++its[k];
        kcols[k] = done;
        est[k] = hd->bstat[k * 4 + 0] / bnorm[k];
        if (its[k] == CF_WARMUP) est_w[k] = est[k];
        if (est[k] <= tol || its[k] >= hd->opt.maxit || hd->bstat[k * 4 + 1] == 0.0) stopped[k] = 1;
        all_stopped = all_stopped && stopped[k];
      }
      return all_stopped ? VH_ENOCONV : VH_OK;  // VH_ENOCONV here: every source stopped
    };
    bool finished = false;
    // complex64 preconditioner: pass B leaves the next input already rounded in bq[0]
    cpx<float>* lo = hd->prec == PREC_F32 ? (cpx<float>*)hd->bq[0] : nullptr;
    for (int j = 0; j < m && !finished; ++j) {
      const void* qv = Vj(j);
      if (hd->prec != PREC_F64) {
        if (j == 0) {
          count(hd, dNS, 16.0 + hd->esz);
          VH_HIP(convert(Vj(j), PREC_F64, hd->bq[0], hd->prec, (size_t)N * S, s));
        }
        qv = hd->bq[0];
      }
      const int tk = hd->tbegin(2);
      VH_TRY(vcycle_b(hd, 0, ls, qv, Zj(j), true));
      hd->tend(tk);
      count(hd, (double)N, 16.0 * k0 + S * (hd->esz + 16.0));
      VH_HIP(batch_stencil(hd->dim, hd->L[0].shape, g0, ls, OP_APPLY, PREC_F64, hd->Hfine, hd->prec, Zj(j),
                           PREC_F64, nullptr, Vj(j + 1), s, hd->L[0].s64_stile));
      count(hd, dNS, 16.0 * (2 * j + 6) + (lo ? 8.0 : 0.0));  // passes A and B
      VH_HIP(batch_dcgs_a(hd->bV, ldv, j, j + 1, N, ls, hd->bpart, hd->bnred, K, s));
      VH_HIP(batch_dcgs_fin(K, j, S, 0, s));
      if (j >= 1) VH_TRY(status_post(hd, hd->bK->status, (size_t)S * 4 * sizeof(double), hd->bstat));
      VH_HIP(batch_dcgs_b(hd->bV, ldv, j, N, ls, K, lo, s));
      if (j >= 1) {
        const vh_status a = account(j, true);
        if (a == VH_ENOCONV) {
          finished = true;
          break;
        }
        VH_TRY(a);
      }
    }
    if (!finished) {
      count(hd, dNS, 16.0 * (m + 2));
      VH_HIP(batch_dcgs_a(hd->bV, ldv, m, m, N, ls, hd->bpart, hd->bnred, K, s));
      VH_HIP(batch_dcgs_fin(K, m, S, 1, s));
      const vh_status a = account(m, false);
      if (a != VH_ENOCONV) VH_TRY(a);
    }
    VH_HIP(hipMemcpyAsync(K->kcols, kcols, S * sizeof(int), hipMemcpyHostToDevice, s));
    int kmax = 0;
    for (int k = 0; k < S; ++k) kmax = kcols[k] > kmax ? kcols[k] : kmax;
    VH_HIP(batch_backsolve(K, S, s));
    count(hd, dNS, (double)kmax * hd->esz + 32.0);
    VH_HIP(batch_update_x(K, kmax, hd->prec, hd->bZ, ldv, hd->bX, N, ls, s));
    count(hd, (double)N, 16.0 * k0 + S * 48.0 + 48.0 * S);  // true residual, norm and scale
    VH_HIP(batch_stencil(hd->dim, hd->L[0].shape, g0, ls, OP_RESID, PREC_F64, hd->Hfine, PREC_F64, hd->bX,
                         PREC_F64, hd->bQ, Vj(0), s, hd->L[0].s64_stile));
    VH_HIP(batch_cgs(2, hd->bV, ldv, 0, K->h2, Vj(0), N, ls, hd->bpart, hd->bnred, K->nrm2, s));
    VH_HIP(batch_cycle_init(K, m, S, s));
    VH_HIP(batch_scale(K, Vj(0), Vj(0), N, ls, s));
    VH_TRY(read_bstatus(hd, S));
    for (int k = 0; k < S; ++k) {
      if (!active[k]) continue;
      beta[k] = hd->bstat[k * 4 + 3];
      ++restarts[k];
      if (!(beta[k] == beta[k]) || std::isinf(beta[k])) return fail(VH_EBREAKDOWN, "non-finite residual");
    }
  }
  count(hd, dNS, 32.0);
  VH_HIP(batch_scatter(N, S, nsrc, hd->bX, u, s));
  VH_HIP(hipStreamSynchronize(s));
  bool all_conv = true;
  for (int k = 0; k < nsrc; ++k) {
    if (st) {
      st[k] = vh_solve_stats{};
      st[k].iterations = its[k];
      st[k].restarts = restarts[k];
      st[k].converged = conv[k];
      st[k].relres = bnorm[k] > 0 ? beta[k] / bnorm[k] : 0.0;
      st[k].relres_est = est[k];
      st[k].c_f = its[k] > CF_WARMUP && est_w[k] > 0.0
                      ? std::pow(est[k] / est_w[k], 1.0 / (its[k] - CF_WARMUP))
                      : NAN;
    }
    all_conv = all_conv && conv[k];
  }
  return all_conv ? VH_OK : fail(VH_ENOCONV, "maxit reached before tol");
}

// ---------------------------------------------------------------- setup
// Geometry of the slabs in which the assembled smoother of a level is built: slabs are
// runs of whole planes of the outermost axis (z in 3D, y in 2D).  The per-patch rows
// of a slab of SZ output planes need the patches centred on SZ + 2 planes, whose
// members span SZ + 4 planes.
struct SlabPlan {
  long long n_out, plane, plane_pad, SZ, cnt_max;
  size_t per_plane;  // bytes of per-patch rows per plane
  bool own;          // true: a temporary buffer, false: the caller's scratch area
};

SlabPlan slab_plan(int dim, const Grid& g, int Np, size_t esz, size_t scratch_bytes) {
  SlabPlan p;
  p.n_out = dim == 3 ? g.nz : g.ny;
  p.plane = dim == 3 ? (long long)g.nx * g.ny : g.nx;
  p.plane_pad = dim == 3 ? (long long)g.nxp * g.ny : g.nxp;
  p.per_plane = (size_t)Np * Np * (size_t)p.plane_pad * esz;
  p.SZ = (long long)(scratch_bytes / p.per_plane) - 4;
  p.own = false;
  if (p.SZ < 8 && p.SZ < p.n_out) {  // scratch too small: up to 16 planes at a time
    p.SZ = p.n_out < 16 ? p.n_out : 16;
    p.own = true;
  }
  if (p.SZ > p.n_out) p.SZ = p.n_out;
  p.cnt_max = p.SZ + 4 < p.n_out ? p.SZ + 4 : p.n_out;
  return p;
}

// Assembled smoother of level Lv built without holding the level's whole per-patch
// array: each slab of output planes gets its patch inverses in the scratch area (the
// patches centred within one plane of the slab), then its assembled rows.
vh_status assemble_level(vh_handle* hd, Level& Lv, const cpx<double>* A, int Np,
                         void* scratch, size_t scratch_bytes, bool sym, bool nopiv) {
  const int dim = hd->dim;
  const Grid& g = Lv.g;
  hipStream_t s = hd->s;
  const SlabPlan p = slab_plan(dim, g, Np, hd->esz, scratch_bytes);
  void* buf = scratch;
  if (p.own) VH_TRY(hd->alloc(&buf, (size_t)p.cnt_max * p.per_plane, true));
  const size_t gstride = (size_t)p.cnt_max * p.plane_pad;
  const int K5 = dim == 2 ? 25 : 125;
  const int E = sym ? (K5 + 1) / 2 : K5;
  const size_t Npad = (size_t)g.Np;
  // the symmetric sweep reads up to sym_guard entries before the first plane and sym_tail
  // after the last: zero guards
  const size_t guard = sym ? (size_t)sym_guard(g) : 0, tail = sym ? (size_t)sym_tail(g) : 0;
  void* base = nullptr;
  VH_TRY(hd->alloc(&base, ((size_t)E * Npad + guard + tail) * hd->esz));
  VH_HIP(fill(base, (size_t)E * Npad + guard + tail, hd->prec, 0, 0, s));  // row padding stays zero
  Lv.B = (char*)base + guard * hd->esz;
  for (long long p0 = 0; p0 < p.n_out; p0 += p.SZ) {
    const long long p1 = p0 + p.SZ < p.n_out ? p0 + p.SZ : p.n_out;
    const long long b0 = p0 - 2 > 0 ? p0 - 2 : 0;
    const long long c0 = p0 - 1 > 0 ? p0 - 1 : 0, c1 = p1 + 1 < p.n_out ? p1 + 1 : p.n_out;
    VH_HIP(vanka_setup(dim, Lv.shape, Lv.patch, g, A, Lv.w, hd->prec, buf,
                       Slab{c0 * p.plane, c1 * p.plane, b0 * p.plane_pad, gstride}, s, nopiv));
    const Slab so{p0 * p.plane, p1 * p.plane, b0 * p.plane_pad, gstride};
    if (sym)
      VH_HIP(vanka_assemble_sym(dim, g, hd->prec, buf, so, Lv.w, Lv.B, s));
    else
      VH_HIP(vanka_assemble(dim, Lv.patch, g, hd->prec, buf, so, Lv.B, s));
  }
  if (p.own) {
    VH_HIP(hipStreamSynchronize(s));
    hd->release(buf);
  }
  Lv.E = E;
  return VH_OK;
}

vh_status build(vh_handle* hd, const double* kappa, const double* gamma) {
  const int dim = hd->dim;
  const vh_options& o = hd->opt;
  const int ig = resolve_intergrid(dim, o.intergrid);
  hipStream_t s = hd->s;
  hd->L.resize(hd->levels);
  // grids and transfer plan
  int nn[3] = {hd->n[0], hd->n[1], dim == 3 ? hd->n[2] : 1};
  int shape = o.stencil == VH_STENCIL_COMPACT4 ? BOX1 : CROSS;
  for (int l = 0; l < hd->levels; ++l) {
    Level& Lv = hd->L[l];
    Lv.g = make_grid(dim, nn[0], nn[1], nn[2]);
    Lv.shape = shape;
    Lv.K = shape_points(dim, shape);
    Lv.patch = (l == 0 && o.fine_patch >= 0) ? o.fine_patch : hd->patch;
    Lv.w = (l < o.ndamping) ? o.damping[l]
                            : (o.ndamping > 0 ? o.damping[o.ndamping - 1]
                                              : default_damping(dim, Lv.patch, l, o.stencil));
    if (l + 1 < hd->levels) {
      int sout;
      VH_TRY(transfer_plan(dim, ig, l, shape, &Lv.rf, &Lv.pf, &sout));
      shape = sout;
      for (int d = 0; d < dim; ++d) nn[d] = (nn[d] - 1) / 2 + 1;
    }
  }
  const size_t N0 = (size_t)hd->L[0].g.N;
  {  // media check: kappa > 0 and gamma >= 0, all finite
    int* flag = nullptr;
    VH_TRY(hd->alloc((void**)&flag, sizeof(int), true));
    VH_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    VH_HIP(check_media((long long)N0, kappa, gamma, flag, s));
    int hflag = 0;
    VH_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    VH_HIP(hipStreamSynchronize(s));
    hd->release(flag);
    if (hflag) return fail(VH_EINVAL, "kappa must be finite and > 0, gamma finite and >= 0");
  }
  // finest operator, FP64
  std::vector<cpx<double>*> A64(hd->levels, nullptr);
  VH_TRY(hd->alloc((void**)&hd->Hfine, hd->L[0].K * N0 * sizeof(cpx<double>)));
  // the FP64 Galerkin operators are the levels' operators in FP64, set-up temporaries
  // when the preconditioner runs in complex64
  const bool a64_temp = hd->prec != PREC_F64;
  VH_TRY(hd->alloc((void**)&A64[0], hd->L[0].K * N0 * sizeof(cpx<double>), a64_temp));
  if (o.stencil == VH_STENCIL_COMPACT4)
    VH_HIP(fine_compact4(dim, hd->L[0].g, kappa, gamma, hd->h, hd->omega, hd->shift, o.bc,
                         o.sponge_width, o.sponge_amp, hd->Hfine, A64[0], s));
  else
    VH_HIP(fine_operator(dim, hd->L[0].g, kappa, gamma, hd->h, hd->omega, hd->shift, o.bc,
                         o.sponge_width, o.sponge_amp, hd->Hfine, A64[0], s));
  if (o.stencil != VH_STENCIL_COMPACT4) {
    // every later application of the 5/7-point operator reads only its centre entries
    hd->L[0].g.offrule = o.bc == VH_BC_ABC ? 2 : 1;
    hd->L[0].g.ih2 = 1.0 / (hd->h * hd->h);
  }
  // Galerkin hierarchy, FP64
  for (int l = 0; l + 1 < hd->levels; ++l) {
    Level &Lf = hd->L[l], &Lc = hd->L[l + 1];
    VH_TRY(hd->alloc((void**)&A64[l + 1], (size_t)Lc.K * Lc.g.N * sizeof(cpx<double>), a64_temp));
    VH_HIP(galerkin(dim, Lf.shape, Lc.shape, Lf.rf, Lf.pf, Lf.g, Lc.g, A64[l], A64[l + 1], s));
  }
  // the FGMRES basis is allocated first: until the first solve it is the scratch
  // area in which the assembled smoother is built slab by slab
  hd->m = o.restart;
  VH_TRY(hd->alloc((void**)&hd->V, (size_t)(hd->m + 1) * N0 * sizeof(cpx<double>)));
  // per level: operator at the preconditioner precision, patch inverses, vectors
  bool sym_above = true;
  for (int l = 0; l < hd->levels; ++l) {
    Level& Lv = hd->L[l];
    const size_t N = (size_t)Lv.g.N;
    if (hd->prec == PREC_F64) {
      Lv.A = A64[l];
    } else {
      VH_TRY(hd->alloc(&Lv.A, (size_t)Lv.K * N * hd->esz));
      VH_HIP(convert(A64[l], PREC_F64, Lv.A, hd->prec, (size_t)Lv.K * N, s));
    }
    VH_TRY(hd->alloc(&Lv.q, N * hd->esz));
    VH_TRY(hd->alloc(&Lv.u, N * hd->esz));
    VH_TRY(hd->alloc(&Lv.r, N * hd->esz));
    VH_HIP(fill(Lv.q, N, hd->prec, 0, 0, s));
    VH_HIP(fill(Lv.u, N, hd->prec, 0, 0, s));
    VH_HIP(fill(Lv.r, N, hd->prec, 0, 0, s));
    Lv.bytes = ((size_t)Lv.K + 3) * N * hd->esz;
    if (l + 1 == hd->levels) break;
    const size_t Npad = (size_t)Lv.g.Np;  // smoother arrays use the padded row layout
    const int Np = patch_size(dim, Lv.patch);
    // H_s^l is symmetric when H_s is and every transfer above level l has R and P of
    // one family (R = c P^T); below a mixed transfer the full stencil is kept
    sym_above = sym_above && (l == 0 || (hd->L[l - 1].rf == hd->L[l - 1].pf));
    // patch matrices of a complex symmetric H_s^l (5/7-point operator) whose imaginary part
    // is positive definite (shift > 0; omega = 0 leaves the Laplacian, positive definite):
    // elimination without pivoting (vh_options.setup_pivot = 1 keeps partial pivoting)
    Lv.nopiv = o.setup_pivot == 0 && sym_above && o.stencil == VH_STENCIL_FD2 &&
               Lv.patch == VH_PATCH_FULL && (hd->shift > 0.0 || hd->omega == 0.0);
    if ((o.smoother == VH_SMOOTHER_ASSEMBLED || o.smoother == VH_SMOOTHER_SYMMETRIC) &&
        Lv.patch != VH_PATCH_POINT) {
      const bool sym = o.smoother == VH_SMOOTHER_SYMMETRIC && sym_above;
      VH_TRY(assemble_level(hd, Lv, A64[l], Np, hd->V, (size_t)(hd->m + 1) * N0 * sizeof(cpx<double>),
                            sym, Lv.nopiv));
      Lv.form = sym ? SM_SYMHALF : 2;
      if (sym && dim == 3) {
        Lv.sym_planes = o.sym_planes == 0 ? sym_walk_planes(Lv.g) : o.sym_planes;
        const size_t nc = (size_t)sym_carry_elems(Lv.g, Lv.sym_planes);
        if (nc) {
          VH_TRY(hd->alloc(&Lv.carry, nc * hd->esz));
          Lv.bytes += nc * hd->esz;
        }
      }
    } else {
      VH_TRY(hd->alloc(&Lv.B, (size_t)Np * Np * Npad * hd->esz));
      VH_HIP(fill(Lv.B, (size_t)Np * Np * Npad, hd->prec, 0, 0, s));
      VH_HIP(vanka_setup(dim, Lv.shape, Lv.patch, Lv.g, A64[l], Lv.w, hd->prec, Lv.B,
                         Slab{0, (long long)N, 0, Npad}, s, Lv.nopiv));
      Lv.E = Np * Np;
      Lv.form = Lv.patch;
    }
    Lv.bytes += (size_t)Lv.E * Npad * hd->esz;
  }
  if (o.smoother == VH_SMOOTHER_ASSEMBLED && hd->patch == VH_PATCH_POINT)
    hd->opt.smoother = VH_SMOOTHER_PATCH;  // a 1x1 patch is already a 1-point stencil
  // coarsest: dense FP64 inverse
  {
    Level& Lc = hd->L[hd->levels - 1];
    const int nc = (int)Lc.g.N;
    hd->nc = nc;
    void* work = nullptr;
    VH_TRY(hd->alloc((void**)&hd->Dinv, (size_t)nc * nc * sizeof(cpx<double>)));
    VH_TRY(hd->alloc(&work, gj_workspace_bytes(nc), true));
    VH_HIP(fill(hd->Dinv, (size_t)nc * nc, PREC_F64, 0, 0, s));
    VH_HIP(dense_assemble(dim, Lc.shape, Lc.g, A64[hd->levels - 1], hd->Dinv, s));
    VH_HIP(gj_invert(nc, hd->Dinv, work, s));
    VH_HIP(hipStreamSynchronize(s));
    hd->release(work);
  }
  VH_HIP(hipStreamSynchronize(s));
  if (hd->prec != PREC_F64)
    for (int l = 0; l < hd->levels; ++l) {
      hd->release(A64[l]);
    }
  // FGMRES workspace (the basis V is already allocated)
  {
    long long nb = (long long)N0 / 512;
    hd->nred = (int)(nb < 64 ? 64 : (nb > 2048 ? 2048 : nb));
  }
  VH_TRY(hd->alloc(&hd->Z, (size_t)hd->m * N0 * hd->esz));
  VH_TRY(hd->alloc((void**)&hd->part, (size_t)hd->nred * 65 * sizeof(cpx<double>)));
  VH_TRY(hd->alloc((void**)&hd->K, sizeof(KrylovDev)));
  VH_HIP(hipMemsetAsync(hd->K, 0, sizeof(KrylovDev), s));
  hd->dnb = hd->nred < 1024 ? hd->nred : 1024;
  VH_TRY(hd->alloc((void**)&hd->dpart, ((size_t)hd->dnb + 16) * 65 * 64 * sizeof(cpx<double>)));
  VH_TRY(hd->alloc((void**)&hd->dK, sizeof(BatchKrylovDev)));
  VH_HIP(hipMemsetAsync(hd->dK, 0, sizeof(BatchKrylovDev), s));
  if (hd->pinned_ext)
    hd->hstat = hd->pinned_ext;
  else
    VH_HIP(hipHostMalloc((void**)&hd->hstat, 4 * sizeof(double), hipHostMallocDefault));
  VH_HIP(hipEventCreateWithFlags(&hd->sev, hipEventDisableTiming));
  if (o.timing) {
    hd->ev.assign(128, nullptr);
    hd->ev_kind.assign(64, 0);
    for (auto& e : hd->ev) VH_HIP(hipEventCreate(&e));
  }
  VH_TRY(tune_fuse(hd));
  VH_HIP(hipStreamSynchronize(s));
  return VH_OK;
}

}  // namespace

// ==================================================================== C ABI
extern "C" {

void vh_options_default(vh_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = VH_PREC_FP64;
  o->restart = 20;
  o->maxit = 1000;
  o->nu1 = 1;
  o->nu2 = 1;
  o->intergrid = -1;
  o->bc = VH_BC_ABC;
  o->sponge_width = 20;
  o->sponge_amp = 1.0;
  o->smoother = VH_SMOOTHER_PATCH;
  o->fine_patch = -1;
  o->ndamping = 0;
  o->stream = nullptr;
}

const char* vh_status_string(vh_status s) {
  switch (s) {
    case VH_OK: return "ok";
    case VH_EINVAL: return "invalid argument";
    case VH_ENOMEM: return "out of device memory";
    case VH_ENOCONV: return "not converged";
    case VH_EBREAKDOWN: return "breakdown (NaN/Inf)";
    case VH_EDEVICE: return "device error";
    case VH_EUNSUPPORTED: return "unsupported option combination";
    default: return "unknown status";
  }
}

const char* vh_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// vh_setup, optionally inside a device region handed over by the caller (see vh_handle)
static vh_status setup_impl(vh_handle** out, int dim, const int* n, double h, double omega,
                            const double* kappa, const double* gamma, double shift, int levels,
                            int patch, const vh_options* opt, void* region, size_t region_bytes,
                            double* pinned) {
  if (!out) return fail(VH_EINVAL, "out is NULL");
  *out = nullptr;
  vh_options o;
  if (opt)
    o = *opt;
  else
    vh_options_default(&o);
  VH_TRY(validate(dim, n, h, omega, shift, levels, patch, o));
  if (!kappa) return fail(VH_EINVAL, "kappa is NULL");
  const int ig = resolve_intergrid(dim, o.intergrid);
  if (ig != VH_IG_LEVDEP && ig != VH_IG_MIXED && ig != VH_IG_LINEAR && ig != VH_IG_CUBIC)
    return fail(VH_EINVAL, "unknown intergrid");
  if (dim == 3 && ig != VH_IG_LINEAR)
    return fail(VH_EUNSUPPORTED, "3D supports only the trilinear intergrid");
  vh_handle* hd = new (std::nothrow) vh_handle();
  if (!hd) return fail(VH_ENOMEM, "host allocation failed");
  hd->dim = dim;
  for (int d = 0; d < dim; ++d) hd->n[d] = n[d];
  hd->h = h;
  hd->omega = omega;
  hd->shift = shift;
  hd->levels = levels;
  hd->patch = patch;
  hd->opt = o;
  hd->prec = o.precision == VH_PREC_FP64 ? PREC_F64 : PREC_F32;
  hd->esz = hd->prec == PREC_F64 ? 16 : 8;
  hd->s = (hipStream_t)o.stream;
  if (region) {
    hd->region = (char*)region;
    hd->region_bytes = region_bytes;
    hd->lo = 0;
    hd->hi = region_bytes;
  }
  hd->pinned_ext = pinned;
  const auto t0 = std::chrono::steady_clock::now();
  vh_status st = build(hd, kappa, gamma);
  hd->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st != VH_OK) {
    (void)hipStreamSynchronize(hd->s);
    delete hd;
    return st;
  }
  *out = hd;
  return VH_OK;
}

vh_status vh_setup_region(vh_handle** out, int dim, const int* n, double h, double omega,
                          const double* kappa, const double* gamma, double shift, int levels,
                          int patch, const vh_options* opt, void* region, size_t region_bytes,
                          double* pinned) {
  if (!region || region_bytes == 0 || !pinned) return fail(VH_EINVAL, "bad region");
  return setup_impl(out, dim, n, h, omega, kappa, gamma, shift, levels, patch, opt, region,
                    region_bytes, pinned);
}

extern "C" {

vh_status vh_setup(vh_handle** out, int dim, const int* n, double h, double omega,
                   const double* kappa, const double* gamma, double shift, int levels, int patch,
                   const vh_options* opt) {
  return setup_impl(out, dim, n, h, omega, kappa, gamma, shift, levels, patch, opt, nullptr, 0,
                    nullptr);
}

vh_status vh_solve(vh_handle* hd, const void* q, int nsrc, double tol, void* u,
                   vh_solve_stats* stats) {
  if (!hd || !q || !u) return fail(VH_EINVAL, "NULL argument");
  if (nsrc < 1) return fail(VH_EINVAL, "nsrc must be >= 1");
  if (!(tol > 0)) return fail(VH_EINVAL, "tol must be > 0");
  if (q == u) return fail(VH_EINVAL, "q and u may not alias");
  const size_t N = (size_t)hd->L[0].g.N;
  vh_status worst = VH_OK;
  if (hd->opt.batch) {
    for (int s0 = 0; s0 < nsrc; s0 += 64) {
      const int cnt = nsrc - s0 < 64 ? nsrc - s0 : 64;
      hipEvent_t e0, e1;
      VH_HIP(hipEventCreate(&e0));
      VH_HIP(hipEventCreate(&e1));
      VH_HIP(hipEventRecord(e0, hd->s));
      for (int k = 0; k < 3; ++k) {
        hd->t_ms[k] = 0;
        hd->t_n[k] = 0;
      }
      hd->ev_used = 0;
      hd->moved = 0.0;
      vh_status r = fgmres_batch(hd, (const cpx<double>*)q + (size_t)s0 * N, cnt,
                                 (cpx<double>*)u + (size_t)s0 * N, tol, stats ? stats + s0 : nullptr);
      (void)hipEventRecord(e1, hd->s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      hd->tflush();
      if (stats)
        for (int k = s0; k < s0 + cnt; ++k) {
          stats[k].solve_ms = ms;
          stats[k].smooth0_launches = hd->t_n[0];
          stats[k].smooth0_ms = hd->t_ms[0];
          stats[k].smooth1_launches = hd->t_n[1];
          stats[k].smooth1_ms = hd->t_ms[1];
          stats[k].vcycles = hd->t_n[2];
          stats[k].vcycle_ms = hd->t_ms[2];
          stats[k].setup_ms = hd->setup_ms;
          stats[k].bytes_moved = hd->moved;
        }
      if (r != VH_OK && r != VH_ENOCONV) return r;
      if (r == VH_ENOCONV) worst = VH_ENOCONV;
    }
    return worst == VH_OK ? VH_OK : fail(worst, "maxit reached before tol");
  }
  for (int sidx = 0; sidx < nsrc; ++sidx) {
    hipEvent_t e0, e1;
    VH_HIP(hipEventCreate(&e0));
    VH_HIP(hipEventCreate(&e1));
    VH_HIP(hipEventRecord(e0, hd->s));
    vh_solve_stats st{};
    for (int k = 0; k < 3; ++k) {
      hd->t_ms[k] = 0;
      hd->t_n[k] = 0;
    }
    hd->ev_used = 0;
    hd->moved = 0.0;
    vh_status r = fgmres_one(hd, (const cpx<double>*)q + sidx * N, (cpx<double>*)u + sidx * N,
                             tol, &st);
    (void)hipEventRecord(e1, hd->s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st.solve_ms = ms;
    hd->tflush();
    st.smooth0_launches = hd->t_n[0];
    st.smooth0_ms = hd->t_ms[0];
    st.smooth1_launches = hd->t_n[1];
    st.smooth1_ms = hd->t_ms[1];
    st.vcycles = hd->t_n[2];
    st.vcycle_ms = hd->t_ms[2];
    st.setup_ms = hd->setup_ms;
    st.bytes_moved = hd->moved;
    if (stats) stats[sidx] = st;
    if (r != VH_OK && r != VH_ENOCONV) return r;
    if (r == VH_ENOCONV) worst = VH_ENOCONV;
  }
  return worst == VH_OK ? VH_OK : fail(worst, "maxit reached before tol");
}

vh_status vh_destroy(vh_handle* hd) {
  if (!hd) return VH_OK;
  (void)hipStreamSynchronize(hd->s);
  delete hd;
  return VH_OK;
}

int vh_num_levels(const vh_handle* hd) { return hd ? hd->levels : 0; }

vh_status vh_get_memory(const vh_handle* hd, size_t* in_use, size_t* peak) {
  if (!hd) return fail(VH_EINVAL, "NULL handle");
  if (in_use) *in_use = hd->bytes;
  if (peak) *peak = hd->peak_bytes;
  return VH_OK;
}

vh_status vh_get_level_info(const vh_handle* hd, int level, vh_level_info* info) {
  if (!hd || !info || level < 0 || level >= hd->levels) return fail(VH_EINVAL, "bad level");
  const Level& Lv = hd->L[level];
  std::memset(info, 0, sizeof(*info));
  info->n[0] = Lv.g.nx;
  info->n[1] = Lv.g.ny;
  info->n[2] = Lv.g.nz;
  info->stencil_points = Lv.K;
  // the symmetric half is exported (and counted here) as the full assembled stencil
  info->smoother_entries = Lv.form == SM_SYMHALF ? (hd->dim == 2 ? 25 : 125) : Lv.E;
  shape_offsets(hd->dim, Lv.shape, Lv.K, info->offsets);
  info->bytes = Lv.bytes;
  info->sweep_tile = Lv.s64_tile;
  info->fused_sweep = Lv.fuse_sweep ? 1 : 0;
  info->fused_restrict = Lv.fuse_restrict ? 1 : 0;
  info->setup_pivot = (level + 1 < hd->levels && !Lv.nopiv) ? 1 : 0;
  if (Lv.form == SM_SYMHALF && hd->dim == 3) info->sym_planes = Lv.sym_planes > 0 ? Lv.sym_planes : 0;
  for (int ls = 6; ls >= 0; --ls)
    if (Lv.mfma_txp[ls]) {
      info->mfma_sources = 1 << ls;
      info->mfma_tile = Lv.mfma_txp[ls];
      info->mfma_rows = Lv.mfma_rows[ls];
      break;
    }
  return VH_OK;
}

vh_status vh_apply_operator(vh_handle* hd, int level, int which, const void* x, void* y) {
  if (!hd || !x || !y || level < 0 || level >= hd->levels) return fail(VH_EINVAL, "bad argument");
  Level& Lv = hd->L[level];
  const size_t N = (size_t)Lv.g.N;
  if (which == 0) {
    if (level != 0) return fail(VH_EINVAL, "the unshifted operator exists on level 0 only");
    VH_HIP(stencil(hd->dim, Lv.shape, Lv.g, OP_APPLY, PREC_F64, hd->Hfine, PREC_F64, x, PREC_F64,
                   nullptr, y, hd->s));
  } else if (hd->prec == PREC_F64) {
    VH_HIP(stencil(hd->dim, Lv.shape, Lv.g, OP_APPLY, PREC_F64, Lv.A, PREC_F64, x, PREC_F64,
                   nullptr, y, hd->s));
  } else {
    VH_HIP(convert(x, PREC_F64, Lv.r, hd->prec, N, hd->s));
    VH_HIP(stencil(hd->dim, Lv.shape, Lv.g, OP_APPLY, hd->prec, Lv.A, hd->prec, Lv.r, hd->prec,
                   nullptr, Lv.u, hd->s));
    VH_HIP(convert(Lv.u, hd->prec, y, PREC_F64, N, hd->s));
  }
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

vh_status vh_apply_vcycle(vh_handle* hd, const void* v, void* z) {
  if (!hd || !v || !z) return fail(VH_EINVAL, "bad argument");
  Level& L0 = hd->L[0];
  const size_t N = (size_t)L0.g.N;
  if (hd->prec == PREC_F64) {
    VH_TRY(vcycle(hd, 0, v, z, true));
  } else {
    VH_TRY(precondition(hd, (const cpx<double>*)v, L0.u));
    VH_HIP(convert(L0.u, hd->prec, z, PREC_F64, N, hd->s));
  }
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

vh_status vh_apply_smoother(vh_handle* hd, int level, const void* q, void* u) {
  if (!hd || !q || !u || level < 0 || level + 1 >= hd->levels)
    return fail(VH_EINVAL, "bad argument (the coarsest level has no smoother)");
  Level& Lv = hd->L[level];
  const size_t N = (size_t)Lv.g.N;
  // the step the V-cycle takes on this level: in one launch where the level forms the
  // residual inside its sweep (into the level's residual array, then copied back)
  const bool fs = fuses_sweep(hd, Lv);
  if (hd->prec == PREC_F64) {
    if (fs) {
      VH_TRY(smooth_fused(hd, Lv, q, u, Lv.r));
      VH_HIP(hipMemcpyAsync(u, Lv.r, N * hd->esz, hipMemcpyDeviceToDevice, hd->s));
    } else {
      VH_TRY(residual(hd, Lv, q, u, Lv.r));
      VH_TRY(smooth(hd, Lv, Lv.r, u, false));
    }
  } else {
    VH_HIP(convert(q, PREC_F64, Lv.q, hd->prec, N, hd->s));
    VH_HIP(convert(u, PREC_F64, Lv.u, hd->prec, N, hd->s));
    if (fs) {
      VH_TRY(smooth_fused(hd, Lv, Lv.q, Lv.u, Lv.r));
      VH_HIP(convert(Lv.r, hd->prec, u, PREC_F64, N, hd->s));
    } else {
      VH_TRY(residual(hd, Lv, Lv.q, Lv.u, Lv.r));
      VH_TRY(smooth(hd, Lv, Lv.r, Lv.u, false));
      VH_HIP(convert(Lv.u, hd->prec, u, PREC_F64, N, hd->s));
    }
  }
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

namespace {
int batch_log2(int nsrc) {
  int ls = 0;
  while ((1 << ls) < nsrc) ++ls;
  return ls;
}
// source-major c128 [nsrc][n] -> node-major [n][S] at the preconditioner precision in dst
vh_status to_batch(vh_handle* hd, long long n, int S, int nsrc, const void* src, void* dst) {
  VH_HIP(batch_gather(n, S, nsrc, (const cpx<double>*)src, hd->bQ, hd->s));
  VH_HIP(convert(hd->bQ, PREC_F64, dst, hd->prec, (size_t)n * S, hd->s));
  return VH_OK;
}
vh_status from_batch(vh_handle* hd, long long n, int S, int nsrc, const void* src, void* dst) {
  VH_HIP(convert(src, hd->prec, hd->bX, PREC_F64, (size_t)n * S, hd->s));
  VH_HIP(batch_scatter(n, S, nsrc, hd->bX, (cpx<double>*)dst, hd->s));
  return VH_OK;
}
}  // namespace

vh_status vh_apply_smoother_batch(vh_handle* hd, int level, int nsrc, const void* q, void* u) {
  if (!hd || !q || !u || level < 0 || level + 1 >= hd->levels || nsrc < 1 || nsrc > 64)
    return fail(VH_EINVAL, "bad argument (1 <= nsrc <= 64; the coarsest level has no smoother)");
  const int ls = batch_log2(nsrc), S = 1 << ls;
  VH_TRY(ensure_batch(hd, S));
  VH_TRY(tune_mfma(hd, ls));
  VH_TRY(tune_s64(hd, ls));
  const long long n = hd->L[level].g.N;
  VH_TRY(to_batch(hd, n, S, nsrc, q, hd->bq[level]));
  VH_TRY(to_batch(hd, n, S, nsrc, u, hd->bu[level]));
  VH_TRY(bresidual(hd, level, ls, hd->bq[level], hd->bu[level], hd->br[level]));
  VH_TRY(bsmooth(hd, level, ls, hd->br[level], hd->bu[level], false));
  VH_TRY(from_batch(hd, n, S, nsrc, hd->bu[level], u));
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

vh_status vh_apply_vcycle_batch(vh_handle* hd, int nsrc, const void* v, void* z) {
  if (!hd || !v || !z || nsrc < 1 || nsrc > 64) return fail(VH_EINVAL, "bad argument (1 <= nsrc <= 64)");
  const int ls = batch_log2(nsrc), S = 1 << ls;
  VH_TRY(ensure_batch(hd, S));
  VH_TRY(tune_mfma(hd, ls));
  VH_TRY(tune_s64(hd, ls));
  const long long n = hd->L[0].g.N;
  VH_TRY(to_batch(hd, n, S, nsrc, v, hd->bq[0]));
  VH_TRY(vcycle_b(hd, 0, ls, hd->bq[0], hd->bZ, true));
  VH_TRY(from_batch(hd, n, S, nsrc, hd->bZ, z));
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

vh_status vh_export_level(const vh_handle* hdc, int level, void* coef, void* smoother,
                          void* coarse_inv) {
  vh_handle* hd = const_cast<vh_handle*>(hdc);
  if (!hd || level < 0 || level >= hd->levels) return fail(VH_EINVAL, "bad level");
  Level& Lv = hd->L[level];
  const size_t N = (size_t)Lv.g.N;
  auto copy_out = [&](const void* src, size_t count, void* dst) -> vh_status {
    if (hd->prec == PREC_F64) {
      VH_HIP(hipMemcpyAsync(dst, src, count * 16, hipMemcpyDeviceToHost, hd->s));
    } else {
      void* tmp = nullptr;
      VH_HIP(hipMalloc(&tmp, count * 16));
      hipError_t e = convert(src, hd->prec, tmp, PREC_F64, count, hd->s);
      if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, count * 16, hipMemcpyDeviceToHost, hd->s);
      if (e == hipSuccess) e = hipStreamSynchronize(hd->s);
      (void)hipFree(tmp);
      if (e != hipSuccess) return fail(VH_EDEVICE, hipGetErrorString(e));
    }
    return VH_OK;
  };
  if (coef) VH_TRY(copy_out(Lv.A, (size_t)Lv.K * N, coef));
  if (smoother && Lv.B) {
    const bool sym = Lv.form == SM_SYMHALF;
    const size_t count = (size_t)(sym ? (hd->dim == 2 ? 25 : 125) : Lv.E) * N;
    void* tmp = nullptr;
    VH_HIP(hipMalloc(&tmp, count * 16));
    hipError_t e = sym ? unpad_sym(Lv.g, Lv.w, hd->prec, Lv.B, (cpx<double>*)tmp, hd->s)
                       : unpad(Lv.g, Lv.E, hd->prec, Lv.B, (cpx<double>*)tmp, hd->s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(smoother, tmp, count * 16, hipMemcpyDeviceToHost, hd->s);
    if (e == hipSuccess) e = hipStreamSynchronize(hd->s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(VH_EDEVICE, hipGetErrorString(e));
  }
  if (coarse_inv) {
    if (level != hd->levels - 1) return fail(VH_EINVAL, "coarse_inv only on the coarsest level");
    VH_HIP(hipMemcpyAsync(coarse_inv, hd->Dinv, (size_t)hd->nc * hd->nc * 16,
                          hipMemcpyDeviceToHost, hd->s));
  }
  VH_HIP(hipStreamSynchronize(hd->s));
  return VH_OK;
}

vh_status vh_sample_level(const vh_handle* hdc, int level, int which, int count,
                          const int64_t* nodes, void* out) {
  vh_handle* hd = const_cast<vh_handle*>(hdc);
  if (!hd || level < 0 || level >= hd->levels || count < 1 || !nodes || !out)
    return fail(VH_EINVAL, "bad argument");
  Level& Lv = hd->L[level];
  const void* src = which == 0 ? Lv.A : Lv.B;
  const bool sym = which == 1 && Lv.form == SM_SYMHALF;
  const int E = which == 0 ? Lv.K : (sym ? (hd->dim == 2 ? 25 : 125) : Lv.E);
  if (which != 0 && which != 1) return fail(VH_EINVAL, "which must be 0 or 1");
  if (!src || E == 0) return fail(VH_EINVAL, "this level has no such array");
  for (int k = 0; k < count; ++k)
    if (nodes[k] < 0 || nodes[k] >= Lv.g.N) return fail(VH_EINVAL, "node index out of range");
  long long* dn = nullptr;
  cpx<double>* dout = nullptr;
  VH_HIP(hipMalloc((void**)&dn, (size_t)count * sizeof(long long)));
  hipError_t e = hipMalloc((void**)&dout, (size_t)count * E * sizeof(cpx<double>));
  if (e == hipSuccess)
    e = hipMemcpyAsync(dn, nodes, (size_t)count * sizeof(long long), hipMemcpyHostToDevice, hd->s);
  if (e == hipSuccess)
    e = sym ? sample_sym(Lv.g, Lv.w, hd->prec, count, dn, src, dout, hd->s)
            : sample(Lv.g, E, which == 1, hd->prec, count, dn, src, dout, hd->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dout, (size_t)count * E * sizeof(cpx<double>), hipMemcpyDeviceToHost,
                       hd->s);
  if (e == hipSuccess) e = hipStreamSynchronize(hd->s);
  (void)hipFree(dn);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return fail(VH_EDEVICE, hipGetErrorString(e));
  return VH_OK;
}

// ---------------------------------------------------------------- parameter selection
// The cycle as a stationary solver, x <- x + M^{-1} (q - A x) from x = 0, and the
// convergence factor of eq. (cf) (Sec. 5.1).  The residual lives in basis column 0 and
// the correction in Z column 0; the update x += Z_0 * 1 reuses the FGMRES solution
// update with y = (1).
vh_status vh_mg_iterate(vh_handle* hd, int which, const void* q, void* x, int warmup, int maxit,
                        double tol, double* hist, vh_cf_stats* stats) {
  if (!hd || !q || !x || q == x || (which != 0 && which != 1) || warmup < 0 || maxit < 1 ||
      !(tol >= 0.0))
    return fail(VH_EINVAL, "bad argument");
  if (which == 1 && hd->prec != PREC_F64)
    return fail(VH_EUNSUPPORTED, "the stationary iteration on H_s needs a VH_PREC_FP64 handle");
  Level& L0 = hd->L[0];
  const size_t N = (size_t)L0.g.N;
  KrylovDev* K = hd->K;
  cpx<double>* r = hd->V;
  const void* A = which == 0 ? (const void*)hd->Hfine : L0.A;
  cpx<double>* xd = (cpx<double>*)x;
  const cpx<double> one = cmk(1.0, 0.0);
  VH_HIP(hipMemcpyAsync(K->y, &one, sizeof(one), hipMemcpyHostToDevice, hd->s));
  VH_HIP(hipStreamSynchronize(hd->s));
  VH_HIP(fill(x, N, PREC_F64, 0.0, 0.0, hd->s));
  double rq = 0.0, rw = NAN, rn = 0.0, rel = 0.0;
  int k = 0;
  bool conv = false;
  for (;; ++k) {
    VH_HIP(stencil(hd->dim, L0.shape, L0.g, OP_RESID, PREC_F64, A, PREC_F64, xd, PREC_F64, q, r,
                   hd->s));
    VH_HIP(cgs_pass(2, hd->V, N, 0, K->h2, r, N, hd->part, hd->nred, K->nrm2, hd->s));
    VH_HIP(cycle_init(K, hd->m, hd->s));
    VH_TRY(read_status(hd));
    rn = hd->hstat[3];
    if (k == 0) {
      rq = rn;
      if (rq == 0.0) {
        conv = true;
        rel = 0.0;
        if (hist) hist[0] = 0.0;
        break;
      }
    }
    rel = rn / rq;
    if (hist) hist[k] = rel;
    if (k == warmup) rw = rn;
    if (!std::isfinite(rn)) break;
    if (rel <= tol) {
      conv = true;
      break;
    }
    if (rel > 1e12 || k == maxit) break;
    VH_TRY(precondition(hd, r, hd->Z));
    VH_HIP(update_x(K, 1, hd->prec, hd->Z, N, xd, N, hd->s));
  }
  VH_HIP(hipStreamSynchronize(hd->s));
  if (stats) {
    stats->iterations = k;
    stats->converged = conv ? 1 : 0;
    stats->relres = rel;
    stats->cf = (k > warmup && rw > 0.0 && std::isfinite(rw))
                    ? std::pow(rn / rw, 1.0 / (double)(k - warmup))
                    : NAN;
  }
  return VH_OK;
}

}  // extern "C"

namespace {

// The damping the build would use on each of the first levels-1 levels.
void effective_damping(int dim, int levels, int patch, const vh_options& o, double* w) {
  for (int l = 0; l + 1 < levels && l < 16; ++l) {
    const int pl = (l == 0 && o.fine_patch >= 0) ? o.fine_patch : patch;
    w[l] = (l < o.ndamping) ? o.damping[l]
                            : (o.ndamping > 0 ? o.damping[o.ndamping - 1]
                                              : default_damping(dim, pl, l, o.stencil));
  }
}

struct DeviceVec {
  void* p = nullptr;
  ~DeviceVec() {
    if (p) (void)hipFree(p);
  }
};

// score of one configuration: FGMRES iterations (objective 0) or c_f (objective 1);
// +inf when the configuration breaks down.  Setup errors other than a breakdown are
// returned.
vh_status score_config(int dim, const int* n, double h, double omega, const double* kappa,
                       const double* gamma, double shift, int levels, int patch,
                       const vh_options& o, const void* q, void* x, int objective, int warmup,
                       int maxit, double tol, double* score, vh_cf_stats* cfs) {
  vh_handle* hd = nullptr;
  vh_status st = vh_setup(&hd, dim, n, h, omega, kappa, gamma, shift, levels, patch, &o);
  if (st != VH_OK) return st;
  if (objective == 0) {
    vh_solve_stats ss{};
    st = vh_solve(hd, q, 1, tol, x, &ss);
    if (st == VH_OK)
      *score = ss.iterations;
    else if (st == VH_ENOCONV)
      *score = o.maxit + 1;
    else if (st == VH_EBREAKDOWN)
      *score = INFINITY;
  } else {
    vh_cf_stats cs{};
    st = vh_mg_iterate(hd, 1, q, x, warmup, maxit, tol, nullptr, &cs);
    if (st == VH_OK) {
      if (cs.converged && cs.iterations <= warmup)
        *score = 0.0;
      else
        *score = std::isfinite(cs.cf) ? cs.cf : INFINITY;
      if (cfs) *cfs = cs;
    }
  }
  const vh_status sd = vh_destroy(hd);
  if (st == VH_ENOCONV || st == VH_EBREAKDOWN) st = VH_OK;
  return st != VH_OK ? st : sd;
}

}  // namespace

extern "C" {

vh_status vh_tune_damping(int dim, const int* n, double h, double omega, const double* kappa,
                          const double* gamma, double shift, int levels, int patch,
                          const vh_options* opt, const void* q, int objective, int warmup,
                          int maxit, double tol, int nw, const double* w, double* damping,
                          double* scores) {
  if (!n || !kappa || !q || !w || !damping || nw < 1 || levels < 2 || levels > 16 ||
      (objective != 0 && objective != 1) || warmup < 0 || maxit < 1 || !(tol > 0.0) ||
      (dim != 2 && dim != 3))
    return fail(VH_EINVAL, "bad argument");
  for (int j = 0; j < nw; ++j)
    if (!std::isfinite(w[j])) return fail(VH_EINVAL, "non-finite damping candidate");
  vh_options o;
  if (opt)
    o = *opt;
  else
    vh_options_default(&o);
  if (objective == 1) o.precision = VH_PREC_FP64;
  if (objective == 0) o.maxit = maxit;
  o.timing = 0;
  double cur[16] = {0};
  effective_damping(dim, levels, patch, o, cur);
  long long N = 1;
  for (int d = 0; d < dim; ++d) N *= (n[d] > 0 ? n[d] : 0);
  if (N <= 0) return fail(VH_EINVAL, "bad grid");
  DeviceVec x;
  VH_HIP(hipMalloc(&x.p, (size_t)N * sizeof(cpx<double>)));
  bool all_ok = true;
  for (int l = 0; l + 1 < levels; ++l) {
    double best = INFINITY;
    int bj = -1;
    for (int j = 0; j < nw; ++j) {
      cur[l] = w[j];
      o.ndamping = levels - 1;
      for (int i = 0; i + 1 < levels; ++i) o.damping[i] = cur[i];
      double sc = INFINITY;
      VH_TRY(score_config(dim, n, h, omega, kappa, gamma, shift, levels, patch, o, q, x.p,
                          objective, warmup, maxit, tol, &sc, nullptr));
      if (scores) scores[(size_t)l * nw + j] = sc;
      if (sc < best) {
        best = sc;
        bj = j;
      }
    }
    if (bj < 0) all_ok = false;
    cur[l] = bj >= 0 ? w[bj] : w[0];
    damping[l] = cur[l];
  }
  return all_ok ? VH_OK : fail(VH_ENOCONV, "every candidate broke down on some level");
}

vh_status vh_tune_shift(int dim, const int* n, double h, double omega, const double* kappa,
                        const double* gamma, int levels, int patch, const vh_options* opt,
                        const void* q, int na, const double* alphas, int warmup, int maxit,
                        double tol, double* alpha, double* cfs) {
  if (!n || !kappa || !q || !alphas || !alpha || na < 1 || warmup < 0 || maxit < 1 ||
      !(tol > 0.0) || (dim != 2 && dim != 3))
    return fail(VH_EINVAL, "bad argument");
  vh_options o;
  if (opt)
    o = *opt;
  else
    vh_options_default(&o);
  o.precision = VH_PREC_FP64;
  o.timing = 0;
  long long N = 1;
  for (int d = 0; d < dim; ++d) N *= (n[d] > 0 ? n[d] : 0);
  if (N <= 0) return fail(VH_EINVAL, "bad grid");
  DeviceVec x;
  VH_HIP(hipMalloc(&x.p, (size_t)N * sizeof(cpx<double>)));
  if (cfs)
    for (int j = 0; j < na; ++j) cfs[j] = NAN;
  for (int j = 0; j < na; ++j) {
    if (!(alphas[j] >= 0.0) || !std::isfinite(alphas[j]))
      return fail(VH_EINVAL, "shift candidates must be finite and >= 0");
    double sc = INFINITY;
    vh_cf_stats cs{};
    cs.cf = NAN;
    VH_TRY(score_config(dim, n, h, omega, kappa, gamma, alphas[j], levels, patch, o, q, x.p, 1,
                        warmup, maxit, tol, &sc, &cs));
    if (cfs) cfs[j] = cs.cf;
    if (sc < 1.0) {
      *alpha = alphas[j];
      return VH_OK;
    }
  }
  return fail(VH_ENOCONV, "no candidate shift gives a convergent cycle");
}

size_t vh_footprint_bytes(int dim, const int* n, int levels, int patch, int nsrc,
                          const vh_options* opt) {
  // Device bytes of build() and vh_solve, allocation by allocation, as the larger of the
  // setup peak (with the FP64 Galerkin copies of a complex64 hierarchy, the temporary slab
  // buffer and the coarsest pivoting arrays) and the solve peak (with the FGMRES
  // workspace and, for opt->batch, the multi-source workspace).
  vh_options o;
  if (opt)
    o = *opt;
  else
    vh_options_default(&o);
  if ((dim != 2 && dim != 3) || !n || levels < 1 || nsrc < 1) return 0;
  for (int d = 0; d < dim; ++d)
    if (n[d] < 3) return 0;
  const size_t esz = o.precision == VH_PREC_FP64 ? 16 : 8;
  const bool c64 = esz != 16;
  const int ig = resolve_intergrid(dim, o.intergrid);
  const int Np_c = patch_size(dim, patch);
  size_t nn[3] = {(size_t)n[0], (size_t)n[1], dim == 3 ? (size_t)n[2] : 1};
  const size_t N0 = nn[0] * nn[1] * nn[2];
  size_t common = 0, a64 = 0, slab_tmp = 0, coarse_tmp = 0;
  int shape = o.stencil == VH_STENCIL_COMPACT4 ? BOX1 : CROSS;
  common += (size_t)shape_points(dim, shape) * N0 * 16;  // unshifted H
  common += (size_t)(o.restart + 1) * N0 * 16;           // FGMRES basis (slab scratch in setup)
  bool sym_above = true;  // H_s^l symmetric (every transfer above with R = c P^T)
  for (int l = 0; l < levels; ++l) {
    const size_t N = nn[0] * nn[1] * nn[2];
    const int K = shape_points(dim, shape);
    // the FP64 Galerkin operator is the level's operator (FP64) or a setup copy (c64)
    if (c64) a64 += (size_t)K * N * 16;
    common += (size_t)K * N * esz + 3 * N * esz;
    if (l + 1 == levels) {
      common += N * N * 16;                                   // coarsest inverse
      coarse_tmp = gj_workspace_bytes((int)N);  // pivots, row map, second copy, panel
      break;
    }
    const int lp = (l == 0 && o.fine_patch >= 0) ? o.fine_patch : patch;
    const int Np = (l == 0 && o.fine_patch >= 0) ? patch_size(dim, lp) : Np_c;
    const bool assembled =
        (o.smoother == VH_SMOOTHER_ASSEMBLED || o.smoother == VH_SMOOTHER_SYMMETRIC) &&
        lp != VH_PATCH_POINT;
    const int K5 = dim == 2 ? 25 : 125;
    const bool sym = assembled && o.smoother == VH_SMOOTHER_SYMMETRIC && sym_above;
    const int E = assembled ? (sym ? (K5 + 1) / 2 : K5) : Np * Np;
    const Grid g = make_grid(dim, (int)nn[0], (int)nn[1], (int)nn[2]);
    const size_t Npad = (size_t)g.Np;
    common += ((size_t)E * Npad + (sym ? (size_t)(sym_guard(g) + sym_tail(g)) : 0)) * esz;
    if (sym && dim == 3)  // the z walk's carry between chunks of planes
      common += (size_t)sym_carry_elems(g, o.sym_planes == 0 ? sym_walk_planes(g) : o.sym_planes) *
                esz;
    if (assembled) {  // a temporary slab buffer when the basis is too small to hold one
      const SlabPlan p = slab_plan(dim, g, Np, esz, (size_t)(o.restart + 1) * N0 * 16);
      if (p.own && (size_t)p.cnt_max * p.per_plane > slab_tmp) slab_tmp = (size_t)p.cnt_max * p.per_plane;
    }
    shape = (ig == VH_IG_LINEAR) ? BOX1
            : (ig == VH_IG_CUBIC && shape != CROSS && shape != BOX1) ? BOX3 : BOX2;
    sym_above = sym_above && (ig == VH_IG_LINEAR || ig == VH_IG_CUBIC || (ig == VH_IG_LEVDEP && l == 0));
    for (int d = 0; d < dim; ++d) nn[d] = (nn[d] - 1) / 2 + 1;
  }
  if (!c64) a64 = 0;
  // setup: media flag, Galerkin copies, and the larger of a slab buffer (per level) and
  // the coarsest pivoting arrays (allocated after the last slab buffer is freed)
  const size_t setup_extra = sizeof(int) + a64 + std::max(slab_tmp, coarse_tmp);
  // solve: Krylov workspace (partial-sum rows as build() sizes them)
  const size_t nred = std::min<size_t>(std::max<size_t>(N0 / 512, 64), 2048);
  const size_t dnb = std::min<size_t>(nred, 1024);
  size_t solve_extra = (size_t)o.restart * N0 * esz + nred * 65 * 16 + sizeof(KrylovDev) +
                       (dnb + 16) * 65 * 64 * 16 + sizeof(BatchKrylovDev);
  if (o.batch) {  // multi-source workspace for one group of S sources (S = 1 included)
    size_t S = 1;
    while (S < (size_t)(nsrc < 64 ? nsrc : 64)) S *= 2;
    const size_t bnred = std::min<size_t>(std::max<size_t>(N0 * S / 8192, 64), 1024);
    solve_extra += (size_t)(o.restart + 1) * N0 * S * 16 + (size_t)o.restart * N0 * S * esz +
                   2 * N0 * S * 16 + (bnred + 16) * 65 * 64 * 16 + sizeof(BatchKrylovDev);
    size_t m[3] = {(size_t)n[0], (size_t)n[1], dim == 3 ? (size_t)n[2] : 1};
    for (int l = 0; l < levels; ++l) {
      solve_extra += 3 * m[0] * m[1] * m[2] * S * esz;
      for (int d = 0; d < dim; ++d) m[d] = (m[d] - 1) / 2 + 1;
    }
  }
  return common + std::max(setup_extra, solve_extra);
}

}  // extern "C"

size_t vh_region_bytes(int dim, const int* n, int levels, int patch, int nsrc,
                       const vh_options* opt) {
  const size_t fp = vh_footprint_bytes(dim, n, levels, patch, nsrc, opt);
  if (fp == 0 || levels < 1) return 0;
  // every array is rounded up to 256 bytes: at most 24 + 10 per level of them
  return fp + (size_t)(24 + 10 * levels) * 256;
}
