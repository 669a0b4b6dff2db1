// vh_batch.hip -- multi-source (batched right-hand side) kernels.
//
// Many sources share one hierarchy (the paper's many-right-hand-side remark after
// its 3D timings: the setup is amortised over all sources).  Vectors of a batch of
// S sources (S a power of two <= 64) are stored node-major, source-fastest: element
// (node i, source s) at i*S + s.  A wavefront covers 64/S nodes x S sources, so every
// operator coefficient and every patch-inverse entry is loaded once per node and
// broadcast to the S lanes of that node, and neighbour reads are contiguous runs of S
// sources.  Krylov quantities are per source and reduced across the nodes of a block
// with lane shuffles (stride S) and a fixed-order tree: a source's result does not
// depend on the values of the other sources, only (through the summation order) on
// the batch width S.
#include <type_traits>

#include "vh_launch.h"

namespace vh {

namespace {

__device__ __forceinline__ void decode_b(unsigned i, const Grid& g, int& x, int& y, int& z) {
  grid_decode(i, g, x, y, z);
}
__device__ __forceinline__ bool inside_b(const Grid& g, int x, int y, int z) {
  return (unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny && (unsigned)z < (unsigned)g.nz;
}
__device__ __forceinline__ long long lin_b(const Grid& g, int x, int y, int z) {
  return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}
__device__ __forceinline__ long long linp_b(const Grid& g, int x, int y, int z) {
  return (long long)x + (long long)g.nxp * ((long long)y + (long long)g.ny * z);
}
inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define VHB_CHECK()                             \
  do {                                          \
    hipError_t e__ = hipGetLastError();         \
    if (e__ != hipSuccess) return e__;          \
  } while (0)

// (node, source) of this thread; log2 of S passed as `ls`
__device__ __forceinline__ bool thread_ns(const Grid& g, int ls, unsigned& node, int& s) {
  const unsigned long long t =
      (unsigned long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  node = (unsigned)(t >> ls);
  s = (int)(t & ((1u << ls) - 1u));
  return node < (unsigned long long)g.N;
}

}  // namespace

// q[s][N] (c128) -> Q[N][S] (c128, sources >= nsrc zero); and back
__global__ __launch_bounds__(256) void kb_gather(long long N, int S, int nsrc,
                                                 const cpx<double>* __restrict__ q,
                                                 cpx<double>* __restrict__ Q) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * S) return;
  const long long i = t / S;
  const int s = (int)(t % S);
  Q[t] = s < nsrc ? q[(size_t)s * N + i] : cmk(0.0, 0.0);
}
__global__ __launch_bounds__(256) void kb_scatter(long long N, int S, int nsrc,
                                                  const cpx<double>* __restrict__ X,
                                                  cpx<double>* __restrict__ u) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nsrc) return;
  const int s = (int)(t / N);
  const long long i = t % N;
  u[t] = X[i * S + s];
}
hipError_t batch_gather(long long N, int S, int nsrc, const cpx<double>* q, cpx<double>* Q,
                        hipStream_t st) {
  kb_gather<<<nblk(N * S, 256), 256, 0, st>>>(N, S, nsrc, q, Q);
  VHB_CHECK();
  return hipSuccess;
}
hipError_t batch_scatter(long long N, int S, int nsrc, const cpx<double>* X, cpx<double>* u,
                         hipStream_t st) {
  kb_scatter<<<nblk(N * nsrc, 256), 256, 0, st>>>(N, S, nsrc, X, u);
  VHB_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------ stencil sweep, batched
template <int DIM, int SHAPE, int MODE, class TC, class TX, class TY>
__global__ __launch_bounds__(256) void kb_stencil(Grid g, int ls, const cpx<TC>* __restrict__ A,
                                                  const cpx<TX>* __restrict__ x,
                                                  const cpx<TY>* __restrict__ b,
                                                  cpx<TY>* __restrict__ y) {
  unsigned i;
  int s;
  if (!thread_ns(g, ls, i, s)) return;
  int cx, cy, cz;
  decode_b(i, g, cx, cy, cz);
  constexpr int K = shape_K<DIM, SHAPE>();
  const size_t N = (size_t)g.N;
  const int S = 1 << ls;
  cpx<TC> acc = cmk<TC>(0, 0);
  if (SHAPE == CROSS && g.offrule != 0) {
    // the 5/7-point operator with fixed off-diagonals (the values the fine operator
    // stores, so the result is the same): only the centre coefficient is read
    const int c[3] = {cx, cy, cz}, n[3] = {g.nx, g.ny, g.nz};
    double scale = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (g.offrule == 2 && (c[d] == 0 || c[d] == n[d] - 1)) scale *= 0.5;
    acc = cfma(A[i], ccast<TC>(x[(size_t)i * S + s]), acc);
#pragma unroll
    for (int k = 1; k < K; ++k) {
      const int d = (k - 1) / 2;
      const bool up = ((k - 1) & 1) != 0;
      const int dx = shape_off<DIM, SHAPE>(k, 0), dy = shape_off<DIM, SHAPE>(k, 1),
                dz = shape_off<DIM, SHAPE>(k, 2);
      // a neighbour outside the grid: the node's own value with weight 0 (no branch)
      const bool ok = inside_b(g, cx + dx, cy + dy, cz + dz);
      const bool lo = c[d] == 0, hi = c[d] == n[d] - 1;
      const double wv = (g.offrule == 2 && ((up && lo) || (!up && hi))) ? -2.0 * g.ih2 : -g.ih2;
      const TC ov = ok ? (TC)(scale * wv) : (TC)0;
      const long long j =
          ok ? (long long)i + dx + (long long)g.nx * (dy + (long long)g.ny * dz) : (long long)i;
      const cpx<TC> xv = ccast<TC>(x[(size_t)j * S + s]);
      acc.re = fma(ov, xv.re, acc.re);
      acc.im = fma(ov, xv.im, acc.im);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int dx = shape_off<DIM, SHAPE>(k, 0), dy = shape_off<DIM, SHAPE>(k, 1),
                dz = shape_off<DIM, SHAPE>(k, 2);
      if (inside_b(g, cx + dx, cy + dy, cz + dz)) {
        const long long j = (long long)i + dx + (long long)g.nx * (dy + (long long)g.ny * dz);
        acc = cfma(A[(size_t)k * N + i], ccast<TC>(x[(size_t)j * S + s]), acc);
      }
    }
  }
  const size_t o = (size_t)i * S + s;
  if (MODE == OP_APPLY)
    y[o] = ccast<TY>(acc);
  else if (MODE == OP_RESID)
    y[o] = ccast<TY>(ccast<TC>(b[o]) - acc);
  else
    y[o] = ccast<TY>(ccast<TC>(y[o]) + acc);
}

// 2D, 64 sources, radius-R stencils (CROSS, BOX1: R = 1; BOX2: R = 2): the walk of
// kb_sweep2d_s64 (defined below) applied to the operator: one wavefront = one node x 64
// sources, a block of 4 wavefronts covers 4 rows and walks along x; the (2R+1)^2 window of
// x lives in registers (TC precision), the next column of the block's 4 + 2R rows comes
// through a (2R+1)-slot LDS ring, the K coefficients of the block's nodes are staged in LDS
// 2R+1 columns at a time, and every global load is issued 2R+1 steps before its use.
constexpr int S64_ROWS = 4, S64_TX = 16;

__device__ __forceinline__ void lds_barrier_s() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>)
template <int B, int E, class F>
__device__ __forceinline__ void bstatic_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    bstatic_for<B + 1, E>(f);
  }
}

// 2D, 64 sources, walk without LDS: one wave = one grid row x 64 sources (lane = source)
// walking along x over a strip of columns, for any radius-R stencil applied to 64 sources,
// out = A x (APPLY), b - A x (RESID) or y + A x (ADD): the batched operator and residual
// (A the level operator, [K][N]) and the assembled smoother (A the 5x5 stencil of B,
// [25][Np] in the padded layout: u = B r from zero, u += B r).  Each lane keeps the
// (2R+1) x (2R+1) window of its node in a register ring of 2R+1+P columns: a step loads
// the next column (rows y - R .. y + R) straight from memory P steps before its first use
// (the rows shared with the neighbouring rows' waves come from the caches), together with
// the output operand and the node's K coefficients.  The coefficients are the same for
// all 64 lanes: one load spreads a node's coefficient words over the lanes (lane l holds
// 32-bit word l) and each coefficient is rebuilt from lane reads (SGPR operands of the
// FMAs).  Coefficients that point outside the grid are exact zeros (no patch contains an
// outside node, and the operators' boundary rows have none), so window values there may be
// any finite in-grid value: loads go to clamped in-grid addresses and need no select, and
// the ring turns have no branch, so the loads of later steps stay in flight.  No LDS and no
// barrier: waves run independently.  The entries are summed in the same order as in the
// LDS walks, so both give the same bits.
// LB: instead of lane reads (two per complex coefficient, vector ALU instructions), each
// wave writes its node's coefficient words to a slot of its own in LDS and reads every
// coefficient back as one broadcast LDS read (all lanes one address).  LDS operations of
// one wave complete in order, so no barrier is needed; the FMAs are the same.
template <int SHAPE, int MODE, class TC, class TX, class TY, int P, bool PADG, bool LB = false>
__global__ __launch_bounds__(256) void kb_walk2d_s64(Grid g, int tx, const cpx<TC>* __restrict__ A,
                                                     const cpx<TX>* __restrict__ x,
                                                     const cpx<TY>* __restrict__ b,
                                                     cpx<TY>* __restrict__ y) {
  constexpr int R = shape_radius<2, SHAPE>(), W = 2 * R + 1;
  constexpr int K = shape_K<2, SHAPE>();
  constexpr int RG = W + P;                                // column ring
  constexpr int NW = 2 * K * (int)(sizeof(TC) / 4);        // coefficient words per node
  constexpr int NL = (NW + 63) / 64;                       // coefficient loads per node
  const int nsx = (g.nx + tx - 1) / tx;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int xs = (int)(blk % (unsigned)nsx) * tx;
  const int yr = (int)(blk / (unsigned)nsx) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (yr >= g.ny) return;  // a whole wave; nothing below synchronises
  const int lane = threadIdx.x & 63;
  const int xe = min(xs + tx, g.nx);
  const int nstep = xe - xs + 2 * R;  // step k loads column xs - R + k, outputs xs + k - 2R
  size_t roff[W];                     // offsets of the window rows yr - R .. yr + R (clamped)
#pragma unroll
  for (int d = 0; d < W; ++d)
    roff[d] = (size_t)lin_b(g, 0, min(max(yr - R + d, 0), g.ny - 1), 0) * 64 + lane;
  const size_t ooff = (size_t)lin_b(g, 0, yr, 0) * 64 + lane;
  const size_t cstride = PADG ? (size_t)g.Np : (size_t)g.N;
  const size_t crow = PADG ? (size_t)linp_b(g, 0, yr, 0) : (size_t)lin_b(g, 0, yr, 0);
  // lane l of a coefficient load reads word l (past the last word: word 0)
  const unsigned* Aw = (const unsigned*)A;
  constexpr int WPE = 2 * (int)(sizeof(TC) / 4);  // words per complex coefficient
  size_t woff[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int wd = lane + 64 * q < NW ? lane + 64 * q : 0;
    woff[q] = ((size_t)(wd / WPE) * cstride + crow) * WPE + (size_t)(wd % WPE);
  }
  cpx<TX> c[RG][W];
  cpx<TY> of[RG];
  unsigned gv[RG][NL];
  // LB: one slot of 64 * NL words per wave (the step's coefficients)
  __shared__ unsigned cws[LB ? 4 : 1][LB ? 64 * NL : 1];
  unsigned* cw = cws[LB ? (threadIdx.x >> 6) : 0];
  auto fetch = [&](int k, auto sl) {
    constexpr int SL = decltype(sl)::value;
    const size_t cc = (size_t)min(max(xs - R + k, 0), g.nx - 1) * 64;
#pragma unroll
    for (int d = 0; d < W; ++d) c[SL][d] = x[roff[d] + cc];
    const int xo = max(xs + k - 2 * R, xs);  // output of step k (k >= 2R in use)
    if constexpr (MODE == OP_RESID) of[SL] = b[ooff + (size_t)xo * 64];
    if constexpr (MODE == OP_ADD) of[SL] = y[ooff + (size_t)xo * 64];
#pragma unroll
    for (int q = 0; q < NL; ++q) gv[SL][q] = Aw[woff[q] + (size_t)xo * WPE];
  };
  auto coef = [&](auto ph, auto ei) -> cpx<TC> {
    constexpr int PH = decltype(ph)::value, e = decltype(ei)::value;
    constexpr int w0 = e * WPE;
    if constexpr (LB) {
      return *(const cpx<TC>*)(cw + w0);
    } else if constexpr (sizeof(TC) == 4) {
      cpx<TC> v;
      v.re = __int_as_float(__builtin_amdgcn_readlane((int)gv[PH][w0 / 64], w0 % 64));
      v.im = __int_as_float(__builtin_amdgcn_readlane((int)gv[PH][(w0 + 1) / 64], (w0 + 1) % 64));
      return v;
    } else {
      const int lo0 = __builtin_amdgcn_readlane((int)gv[PH][w0 / 64], w0 % 64);
      const int hi0 = __builtin_amdgcn_readlane((int)gv[PH][(w0 + 1) / 64], (w0 + 1) % 64);
      const int lo1 = __builtin_amdgcn_readlane((int)gv[PH][(w0 + 2) / 64], (w0 + 2) % 64);
      const int hi1 = __builtin_amdgcn_readlane((int)gv[PH][(w0 + 3) / 64], (w0 + 3) % 64);
      return cmk<TC>((TC)__hiloint2double(hi0, lo0), (TC)__hiloint2double(hi1, lo1));
    }
  };
  // step k: fetch the column of step k + P (clamped: past the strip's end it loads in-grid
  // values nobody uses), then (k >= 2R) the output xs + k - 2R
  auto step = [&](int k, auto ph, bool out) {
    constexpr int PH = decltype(ph)::value;  // k % RG
    fetch(k + P, std::integral_constant<int, (PH + P) % RG>{});
    if (out) {
      const int xo = xs + k - 2 * R;
      if constexpr (LB) {
        // the previous step's broadcast reads were issued before this write (one wave's
        // LDS operations complete in order); the words are read back as complex values,
        // so a compiler barrier keeps those reads after the write
#pragma unroll
        for (int q = 0; q < NL; ++q) cw[lane + 64 * q] = gv[PH][q];
        asm volatile("" ::: "memory");
      }
      cpx<TC> acc = cmk<TC>(0, 0);
      if constexpr (LB) {
        // the broadcast reads go in groups of 5 entries, each group read while the
        // previous one is summed; a compiler barrier between groups keeps the reads from
        // all being hoisted to the top (register pressure)
        constexpr int NG = (K + 4) / 5;
        cpx<TC> cb[2][5];
        auto rd = [&](auto gi) {
          constexpr int G = decltype(gi)::value;
          bstatic_for<0, 5>([&](auto qi) {
            constexpr int e = G * 5 + decltype(qi)::value;
            if constexpr (e < K) cb[G & 1][decltype(qi)::value] = coef(ph, std::integral_constant<int, e>{});
          });
        };
        rd(std::integral_constant<int, 0>{});
        bstatic_for<0, NG>([&](auto gi) {
          constexpr int G = decltype(gi)::value;
          if constexpr (G + 1 < NG) rd(std::integral_constant<int, G + 1>{});
          asm volatile("" ::: "memory");
          bstatic_for<0, 5>([&](auto qi) {
            constexpr int e = G * 5 + decltype(qi)::value;
            if constexpr (e < K) {
              constexpr int dx = shape_off<2, SHAPE>(e, 0), dy = shape_off<2, SHAPE>(e, 1);
              acc = cfma(cb[G & 1][decltype(qi)::value],
                         ccast<TC>(c[(PH + dx - R + 2 * RG) % RG][dy + R]), acc);
            }
          });
        });
      } else {
        bstatic_for<0, K>([&](auto ei) {
          constexpr int e = decltype(ei)::value;
          constexpr int dx = shape_off<2, SHAPE>(e, 0), dy = shape_off<2, SHAPE>(e, 1);
          acc = cfma(coef(ph, ei), ccast<TC>(c[(PH + dx - R + 2 * RG) % RG][dy + R]), acc);
        });
      }
      const size_t o = ooff + (size_t)xo * 64;
      if constexpr (MODE == OP_APPLY)
        y[o] = ccast<TY>(acc);
      else if constexpr (MODE == OP_RESID)
        y[o] = ccast<TY>(ccast<TC>(of[PH]) - acc);
      else
        y[o] = ccast<TY>(ccast<TC>(of[PH]) + acc);
    }
  };
  // the loads of every step are issued unconditionally and the main loop runs whole ring
  // turns without a branch inside; the last partial turn is the only guarded code
  bstatic_for<0, P>([&](auto i) { fetch(i.value, i); });
  bstatic_for<0, 2 * R>([&](auto i) {
    step(i.value, std::integral_constant<int, i.value % RG>{}, false);
  });
  int k0 = 2 * R;
#pragma unroll 1
  for (; k0 + RG <= nstep; k0 += RG)
    bstatic_for<0, RG>([&](auto j) {
      step(k0 + j.value, std::integral_constant<int, (2 * R + j.value) % RG>{}, true);
    });
  bstatic_for<0, RG - 1>([&](auto j) {
    if (k0 + j.value < nstep)
      step(k0 + j.value, std::integral_constant<int, (2 * R + j.value) % RG>{}, true);
  });
}


template <int SHAPE, int MODE, class TC, class TX, class TY>
__global__ __launch_bounds__(256) void kb_stencil2d_s64(Grid g, int tx,
                                                        const cpx<TC>* __restrict__ A,
                                                        const cpx<TX>* __restrict__ x,
                                                        const cpx<TY>* __restrict__ b,
                                                        cpx<TY>* __restrict__ y) {
  constexpr int R = shape_radius<2, SHAPE>(), CH = 2 * R + 1, CR = S64_ROWS + 2 * R;
  constexpr int K = shape_K<2, SHAPE>();
  constexpr int CL = (CR * 64 + 255) / 256;  // column values per thread
  constexpr int GN = S64_ROWS * K * CH, GPT = (GN + 255) / 256;
  __shared__ cpx<TX> col[CH][CR][64];
  __shared__ cpx<TC> gch[2][S64_ROWS][K][CH];
  const int nsx = (g.nx + tx - 1) / tx;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int xs = (int)(blk % (unsigned)nsx) * tx, y0 = (int)(blk / (unsigned)nsx) * S64_ROWS;
  const int xe = min(xs + tx, g.nx);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int yy = y0 + wv;
  const bool row_ok = yy < g.ny;
  const size_t N = (size_t)g.N;
  const size_t orow = (size_t)lin_b(g, 0, row_ok ? yy : 0, 0) * 64 + lane;
  const int nstep = xe - xs + 2 * R;  // step k reads column xs - R + k, outputs xs + k - 2R
  cpx<TC> w[CH][CH];                  // [dy][column ring slot]
  cpx<TX> pc[CH][CL];                 // columns in flight, by ring slot
  cpx<TY> bf[CH];                     // b (RESID) or y (ADD) of the outputs in flight
  cpx<TC> gp[GPT];
  auto fetch_col = [&](int cx, cpx<TX>* dst) {
    const bool xok = (unsigned)cx < (unsigned)g.nx;
#pragma unroll
    for (int c = 0; c < CL; ++c) {
      const int v = (int)threadIdx.x + 256 * c, row = v >> 6;
      const int ry = y0 - R + row;
      dst[c] = (row < CR && xok && (unsigned)ry < (unsigned)g.ny)
                   ? x[(size_t)lin_b(g, cx, ry, 0) * 64 + lane]
                   : cmk<TX>(0, 0);
    }
  };
  auto fetch_out = [&](int xo) -> cpx<TY> {
    if (MODE == OP_APPLY || xo < xs || xo >= xe || !row_ok) return cmk<TY>(0, 0);
    return MODE == OP_RESID ? b[orow + (size_t)xo * 64] : y[orow + (size_t)xo * 64];
  };
  // chunk q: output nodes xs + CH q - 2R + j (j < CH), rows y0 .. y0 + 3, entries [e]
  auto fetch_g = [&](int q) {
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      const int j = idx % CH, e = (idx / CH) % K, row = idx / (CH * K);
      const int xo = xs + CH * q - 2 * R + j, ry = y0 + row;
      gp[i] = (idx < GN && xo >= xs && xo < xe && ry < g.ny)
                  ? A[(size_t)e * N + (size_t)lin_b(g, xo, ry, 0)]
                  : cmk<TC>(0, 0);
    }
  };
  auto store_g = [&](int q) {
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      if (idx < GN) (&gch[q & 1][0][0][0])[idx] = gp[i];
    }
  };
  auto step = [&](int k, auto ph) {
    constexpr int PH = decltype(ph)::value;  // k % CH
#pragma unroll
    for (int c = 0; c < CL; ++c) {
      const int v = (int)threadIdx.x + 256 * c, row = v >> 6;
      if (row < CR) col[PH][row][lane] = pc[PH][c];
    }
    if (k + CH < nstep) fetch_col(xs - R + k + CH, pc[PH]);
    lds_barrier_s();
    if (PH == 0) {
      const int q = k / CH;
      if (CH * (q + 1) < nstep) store_g(q + 1);
      if (CH * (q + 2) < nstep) fetch_g(q + 2);
    }
#pragma unroll
    for (int dy = 0; dy < CH; ++dy) w[dy][PH] = ccast<TC>(col[PH][wv + dy][lane]);
    const cpx<TY> bo = bf[PH];
    if (MODE != OP_APPLY) bf[PH] = fetch_out(xs + k + CH - 2 * R);  // the output of step k + CH
    if (k >= 2 * R && row_ok) {
      const cpx<TC>* gq = &gch[(k / CH) & 1][wv][0][PH];
      cpx<TC> acc = cmk<TC>(0, 0);
#pragma unroll
      for (int e = 0; e < K; ++e) {
        const int dx = shape_off<2, SHAPE>(e, 0), dy = shape_off<2, SHAPE>(e, 1);
        acc = cfma(gq[e * CH], w[dy + R][(PH + dx - R + 2 * CH) % CH], acc);
      }
      const size_t o = orow + (size_t)(xs + k - 2 * R) * 64;
      if (MODE == OP_APPLY)
        y[o] = ccast<TY>(acc);
      else if (MODE == OP_RESID)
        y[o] = ccast<TY>(ccast<TC>(bo) - acc);
      else
        y[o] = ccast<TY>(ccast<TC>(bo) + acc);
    }
  };
#pragma unroll
  for (int p = 0; p < CH; ++p) {
    fetch_col(xs - R + p, pc[p]);
    bf[p] = fetch_out(xs + p - 2 * R);
  }
  fetch_g(0);
  store_g(0);
  fetch_g(1);
#pragma unroll 1
  for (int k0 = 0; k0 < nstep; k0 += CH) {
    step(k0, std::integral_constant<int, 0>{});
    if constexpr (CH > 1) if (k0 + 1 < nstep) step(k0 + 1, std::integral_constant<int, 1 % CH>{});
    if constexpr (CH > 2) if (k0 + 2 < nstep) step(k0 + 2, std::integral_constant<int, 2 % CH>{});
    if constexpr (CH > 3) if (k0 + 3 < nstep) step(k0 + 3, std::integral_constant<int, 3 % CH>{});
    if constexpr (CH > 4) if (k0 + 4 < nstep) step(k0 + 4, std::integral_constant<int, 4 % CH>{});
  }
}

template <int SHAPE, int MODE, class TC, class TX, class TY, int P, bool LB = false>
static void launch_stencil_s64w(Grid g, int tx0, const void* A, const void* x, const void* b,
                                void* y, hipStream_t st) {
  const int nsx = (g.nx + tx0 - 1) / tx0;
  const int tx = (g.nx + nsx - 1) / nsx;
  const int nsx2 = (g.nx + tx - 1) / tx;
  const unsigned nb = (unsigned)nsx2 * (unsigned)((g.ny + 3) / 4);
  kb_walk2d_s64<SHAPE, MODE, TC, TX, TY, P, false, LB><<<nb, 256, 0, st>>>(
      g, tx, (const cpx<TC>*)A, (const cpx<TX>*)x, (const cpx<TY>*)b, (cpx<TY>*)y);
}

template <int SHAPE, int MODE, class TC, class TX, class TY>
static void launch_stencil_s64(Grid g, const void* A, const void* x, const void* b, void* y,
                               hipStream_t st) {
  const int nsx = (g.nx + S64_TX - 1) / S64_TX;
  const int tx = (g.nx + nsx - 1) / nsx;
  const int nsx2 = (g.nx + tx - 1) / tx;
  const unsigned nb = (unsigned)nsx2 * (unsigned)((g.ny + S64_ROWS - 1) / S64_ROWS);
  kb_stencil2d_s64<SHAPE, MODE, TC, TX, TY><<<nb, 256, 0, st>>>(
      g, tx, (const cpx<TC>*)A, (const cpx<TX>*)x, (const cpx<TY>*)b, (cpx<TY>*)y);
}

// 64-source 2D stencil by tile code (as the sweep's: 1 = the LDS walk, 2..7 = the
// independent-wave walk with prefetch 2 or 3 over strips of 16, 32 or 64 columns, 8..10 =
// tiles 5..7 with the coefficients broadcast from LDS instead of lane reads)
template <int SHAPE, int MODE, class TC, class TX, class TY>
static void launch_stencil_s64_tile(int tile, Grid g, const void* A, const void* x, const void* b,
                                    void* y, hipStream_t st) {
  static constexpr int TXS[3] = {16, 32, 64};
  if (tile == 0) tile = S64_DEFAULT_TILE;
  if (tile <= 1 || tile > S64_TILES)
    launch_stencil_s64<SHAPE, MODE, TC, TX, TY>(g, A, x, b, y, st);
  else if (tile <= 4)
    launch_stencil_s64w<SHAPE, MODE, TC, TX, TY, 2>(g, TXS[tile - 2], A, x, b, y, st);
  else if (tile <= 7)
    launch_stencil_s64w<SHAPE, MODE, TC, TX, TY, 3>(g, TXS[tile - 5], A, x, b, y, st);
  else
    launch_stencil_s64w<SHAPE, MODE, TC, TX, TY, 3, true>(g, TXS[tile - 8], A, x, b, y, st);
}

template <int DIM, int SHAPE, class TC, class TX, class TY>
static hipError_t bstencil_t(Grid g, int ls, int mode, const void* A, const void* x, const void* b,
                             void* y, hipStream_t st, int tile) {
  if constexpr (DIM == 2 && SHAPE != BOX3) {
    if (ls == 6) {
      if (mode == OP_APPLY)
        launch_stencil_s64_tile<SHAPE, OP_APPLY, TC, TX, TY>(tile, g, A, x, b, y, st);
      else if (mode == OP_RESID)
        launch_stencil_s64_tile<SHAPE, OP_RESID, TC, TX, TY>(tile, g, A, x, b, y, st);
      else
        launch_stencil_s64_tile<SHAPE, OP_ADD, TC, TX, TY>(tile, g, A, x, b, y, st);
      VHB_CHECK();
      return hipSuccess;
    }
  }
  const unsigned nb = nblk(g.N << ls, 256);
  auto Ap = (const cpx<TC>*)A;
  auto xp = (const cpx<TX>*)x;
  auto bp = (const cpx<TY>*)b;
  auto yp = (cpx<TY>*)y;
  if (mode == OP_APPLY)
    kb_stencil<DIM, SHAPE, OP_APPLY, TC, TX, TY><<<nb, 256, 0, st>>>(g, ls, Ap, xp, bp, yp);
  else if (mode == OP_RESID)
    kb_stencil<DIM, SHAPE, OP_RESID, TC, TX, TY><<<nb, 256, 0, st>>>(g, ls, Ap, xp, bp, yp);
  else
    kb_stencil<DIM, SHAPE, OP_ADD, TC, TX, TY><<<nb, 256, 0, st>>>(g, ls, Ap, xp, bp, yp);
  VHB_CHECK();
  return hipSuccess;
}

template <int DIM, int SHAPE>
static hipError_t bstencil_p(Grid g, int ls, int mode, int pc, const void* A, int px,
                             const void* x, int py, const void* b, void* y, hipStream_t st,
                             int tile) {
  if (pc == PREC_F64 && px == PREC_F64 && py == PREC_F64)
    return bstencil_t<DIM, SHAPE, double, double, double>(g, ls, mode, A, x, b, y, st, tile);
  if (pc == PREC_F32 && px == PREC_F32 && py == PREC_F32)
    return bstencil_t<DIM, SHAPE, float, float, float>(g, ls, mode, A, x, b, y, st, tile);
  if (pc == PREC_F64 && px == PREC_F32 && py == PREC_F64)
    return bstencil_t<DIM, SHAPE, double, float, double>(g, ls, mode, A, x, b, y, st, tile);
  return hipErrorInvalidValue;
}

hipError_t batch_stencil(int dim, int shape, Grid g, int ls, int mode, int pc, const void* A,
                         int px, const void* x, int py, const void* b, void* y, hipStream_t st,
                         int tile) {
  if (dim == 2) {
    if (shape == CROSS) return bstencil_p<2, CROSS>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
    if (shape == BOX1) return bstencil_p<2, BOX1>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
    if (shape == BOX2) return bstencil_p<2, BOX2>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
    if (shape == BOX3) return bstencil_p<2, BOX3>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
  } else {
    if (shape == CROSS) return bstencil_p<3, CROSS>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
    if (shape == BOX1) return bstencil_p<3, BOX1>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
    if (shape == BOX2) return bstencil_p<3, BOX2>(g, ls, mode, pc, A, px, x, py, b, y, st, tile);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ additive Vanka, batched
// u[i][s] (+)= sum_e G[e][i] r[i + d_e][s]: the same gather as the single-source sweep;
// each entry G[e][i] is loaded once per node and used for all S sources.
template <int DIM, int FORM>
__host__ __device__ constexpr int bsm_entries() {
  return FORM == 2 ? shape_K<DIM, BOX2>() : patch_Np<DIM, FORM>() * patch_Np<DIM, FORM>();
}
template <int DIM, int FORM>
__host__ __device__ constexpr int bsm_off(int e, int c) {
  return FORM == 2 ? shape_off<DIM, BOX2>(e, c)
                   : patch_off<DIM, FORM>(e % patch_Np<DIM, FORM>(), c) -
                         patch_off<DIM, FORM>(e / patch_Np<DIM, FORM>(), c);
}

template <int DIM, int FORM, bool ZERO, class T>
__global__ __launch_bounds__(256) void kb_sweep(Grid g, int ls, const cpx<T>* __restrict__ G,
                                                const cpx<T>* __restrict__ r,
                                                cpx<T>* __restrict__ u) {
  unsigned i;
  int s;
  if (!thread_ns(g, ls, i, s)) return;
  int cx, cy, cz;
  decode_b(i, g, cx, cy, cz);
  const long long ip = linp_b(g, cx, cy, cz);
  const size_t Np = (size_t)g.Np;
  const int S = 1 << ls;
  constexpr int E = bsm_entries<DIM, FORM>();
  constexpr int UNR = (DIM == 3 && FORM == 0) ? 27 : (E > 128 ? patch_Np<DIM, FORM>() : E);
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll 1
  for (int e0 = 0; e0 < E; e0 += UNR) {
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const int e = e0 + q;
      const int dx = bsm_off<DIM, FORM>(e, 0), dy = bsm_off<DIM, FORM>(e, 1),
                dz = bsm_off<DIM, FORM>(e, 2);
      if (inside_b(g, cx + dx, cy + dy, cz + dz)) {
        const long long j = (long long)i + dx + (long long)g.nx * (dy + (long long)g.ny * dz);
        acc = cfma(G[(size_t)e * Np + ip], r[(size_t)j * S + s], acc);
      }
    }
  }
  const size_t o = (size_t)i * S + s;
  u[o] = ZERO ? acc : (u[o] + acc);
}

// 2D: one block = one row segment of 256/S nodes x S sources; the residual of the
// segment with a halo of 2 (all S sources) is staged in LDS once, so the Np*Np
// neighbour reads of every (node, source) pair come from LDS.
template <int FORM, bool ZERO, class T>
__global__ __launch_bounds__(256) void kb_sweep2d(Grid g, int ls, const cpx<T>* __restrict__ G,
                                                  const cpx<T>* __restrict__ r,
                                                  cpx<T>* __restrict__ u) {
  extern __shared__ unsigned char smem[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem);
  const int S = 1 << ls, NB = 256 >> ls, SX = NB + 4;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (g.nx + NB - 1) / NB;
  const int x0 = (int)(b % (unsigned)nbx) * NB, y0 = (int)(b / (unsigned)nbx);
  for (int e = threadIdx.x; e < SX * 5 * S; e += 256) {
    const int pos = e >> ls, s = e & (S - 1);
    const int gx = x0 + pos % SX - 2, gy = y0 + pos / SX - 2;
    tile[e] = inside_b(g, gx, gy, 0) ? r[(size_t)lin_b(g, gx, gy, 0) * S + s] : cmk<T>(0, 0);
  }
  __syncthreads();
  const int ns = threadIdx.x >> ls, s = threadIdx.x & (S - 1);
  const int x = x0 + ns, y = y0;
  if (x >= g.nx) return;
  const long long i = lin_b(g, x, y, 0), ip = linp_b(g, x, y, 0);
  const size_t Np = (size_t)g.Np;
  constexpr int E = bsm_entries<2, FORM>();
  const cpx<T>* t0 = tile + ((size_t)(ns + 2) + (size_t)SX * 2) * S + s;
  const cpx<T>* Gn = G + ip;
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int dx = bsm_off<2, FORM>(e, 0), dy = bsm_off<2, FORM>(e, 1);
    acc = cfma(Gn[(size_t)e * Np], t0[(dx + SX * dy) * S], acc);
  }
  const size_t o = (size_t)i * S + s;
  u[o] = ZERO ? acc : (u[o] + acc);
}

// 2D, 16 to 64 sources: a block covers a row segment of 16 nodes x S sources (each
// thread 16*S/256 (node, source) pairs).  With many sources per node, per-lane loads of
// the smoother entries would be 8-byte broadcasts; instead the block stages the
// entries of its 16 nodes in LDS with coalesced 16-node row loads, next to the
// residual tile, and every lane reads its node's entries as LDS broadcasts.
constexpr int BW_NB = 16;

template <int FORM, bool ZERO, class T, int LS>
__global__ __launch_bounds__(256) void kb_sweep2d_wide(Grid g, const cpx<T>* __restrict__ G,
                                                       const cpx<T>* __restrict__ r,
                                                       cpx<T>* __restrict__ u) {
  constexpr int E = bsm_entries<2, FORM>();
  constexpr int NB = BW_NB, SX = NB + 4, S = 1 << LS;
  constexpr int NG = E * NB, NT = SX * 5 * S;
  extern __shared__ unsigned char smem[];
  cpx<T>* gt = reinterpret_cast<cpx<T>*>(smem);  // [E][NB]
  cpx<T>* tile = gt + NG;                         // [SX*5][S]
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int nbx = (g.nx + NB - 1) / NB;
  const int x0 = (int)(b % (unsigned)nbx) * NB, y0 = (int)(b / (unsigned)nbx);
  const size_t Np = (size_t)g.Np;
  const long long ip0 = linp_b(g, x0, y0, 0);
  // all loads of the staging phase are issued before the first LDS write
  cpx<T> gv[(NG + 255) / 256], tv[(NT + 255) / 256];
#pragma unroll
  for (int i = 0; i < (NG + 255) / 256; ++i) {
    const int e = threadIdx.x + 256 * i, k = e % NB, q = e / NB;
    gv[i] = (e < NG && x0 + k < g.nx) ? G[(size_t)q * Np + ip0 + k] : cmk<T>(0, 0);
  }
#pragma unroll
  for (int i = 0; i < (NT + 255) / 256; ++i) {
    const int e = threadIdx.x + 256 * i, pos = e >> LS, sl = e & (S - 1);
    const int gx = x0 + pos % SX - 2, gy = y0 + pos / SX - 2;
    tv[i] = (e < NT && inside_b(g, gx, gy, 0)) ? r[(size_t)lin_b(g, gx, gy, 0) * S + sl]
                                                : cmk<T>(0, 0);
  }
#pragma unroll
  for (int i = 0; i < (NG + 255) / 256; ++i)
    if (threadIdx.x + 256 * i < NG) gt[threadIdx.x + 256 * i] = gv[i];
#pragma unroll
  for (int i = 0; i < (NT + 255) / 256; ++i)
    if (threadIdx.x + 256 * i < NT) tile[threadIdx.x + 256 * i] = tv[i];
  __syncthreads();
  const int s = threadIdx.x & (S - 1);
#pragma unroll 1
  for (int ns = threadIdx.x >> LS; ns < NB; ns += 256 >> LS) {
    const int x = x0 + ns;
    if (x >= g.nx) break;
    const cpx<T>* t0 = tile + ((size_t)(ns + 2) + (size_t)SX * 2) * S + s;
    cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int dx = bsm_off<2, FORM>(e, 0), dy = bsm_off<2, FORM>(e, 1);
      acc = cfma(gt[e * NB + ns], t0[(dx + SX * dy) * S], acc);
    }
    const size_t o = (size_t)lin_b(g, x, y0, 0) * S + s;
    u[o] = ZERO ? acc : (u[o] + acc);
  }
}

// 2D, 64 sources: one wave = one node x 64 sources (lane = source).  A block of 4 waves
// covers 4 grid rows and walks along x over a strip of columns, one column per step.
//  - residual: each lane keeps the 5 x 5 window of its node in registers (a ring over
//    the 5 columns, indexed at compile time by unrolling the walk by 5); a step brings in
//    the next column of the block's 8 residual rows (y0 - 2 .. y0 + 5) through a 5-slot
//    LDS ring, so a residual value is loaded from memory twice per sweep (8 rows for 4
//    outputs) and read from LDS 5 times;
//  - smoother entries: wave-uniform per node, staged in LDS for 5 steps at a time with
//    row-segment loads and read as broadcasts;
//  - every global load is issued 5 steps (or one 5-step chunk) before its use, so the
//    walk does not wait on memory latency at each step.
// One barrier per step: column k is written to ring slot k % 5 before the barrier of
// step k and read after it, its next writer is step k + 5; the entries of chunk q + 1
// are written after the barrier of step 5q (chunk q - 1, the previous user of that
// buffer, was read before it) and first read after the barrier of step 5q + 5.
constexpr int B64_ROWS = 4, B64_TX = 16;


__device__ __forceinline__ void lds_barrier_b() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int FORM, bool ZERO, class T>
__global__ __launch_bounds__(256) void kb_sweep2d_s64(Grid g, int tx,
                                                      const cpx<T>* __restrict__ G,
                                                      const cpx<T>* __restrict__ r,
                                                      cpx<T>* __restrict__ u) {
  constexpr int E = bsm_entries<2, FORM>();
  constexpr int CR = B64_ROWS + 4, CH = 5;
  constexpr int GN = B64_ROWS * E * CH, GPT = (GN + 255) / 256;
  __shared__ cpx<T> col[CH][CR][64];
  __shared__ cpx<T> gch[2][B64_ROWS][E][CH];
  const int nsx = (g.nx + tx - 1) / tx;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int xs = (int)(b % (unsigned)nsx) * tx, y0 = (int)(b / (unsigned)nsx) * B64_ROWS;
  const int xe = min(xs + tx, g.nx);  // outputs xs .. xe - 1
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int y = y0 + wv;
  const bool row_ok = y < g.ny;
  // this thread's two residual rows of every column: y0 - 2 + wv and y0 + 2 + wv
  const int ya = y0 - 2 + wv, yb = y0 + 2 + wv;
  const bool ya_ok = (unsigned)ya < (unsigned)g.ny, yb_ok = (unsigned)yb < (unsigned)g.ny;
  const cpx<T>* ra = r + (size_t)lin_b(g, 0, ya_ok ? ya : 0, 0) * 64 + lane;
  const cpx<T>* rb = r + (size_t)lin_b(g, 0, yb_ok ? yb : 0, 0) * 64 + lane;
  const size_t Np = (size_t)g.Np;
  cpx<T>* ur = u + (size_t)lin_b(g, 0, row_ok ? y : 0, 0) * 64 + lane;
  const int nstep = xe - xs + 4;  // step k reads column xs - 2 + k, outputs xs + k - 4
  cpx<T> w[5][5];                 // [dy][column ring slot]
  cpx<T> pa[CH], pb[CH];          // residual columns in flight, by ring slot
  cpx<T> uf[CH];                  // u of the outputs in flight, by ring slot
  cpx<T> gp[GPT];                 // smoother entries of the next chunk
  auto fetch_col = [&](int cx, cpx<T>& a, cpx<T>& c) {
    const bool ok = (unsigned)cx < (unsigned)g.nx;
    a = (ok && ya_ok) ? ra[(size_t)cx * 64] : cmk<T>(0, 0);
    c = (ok && yb_ok) ? rb[(size_t)cx * 64] : cmk<T>(0, 0);
  };
  auto fetch_u = [&](int x) -> cpx<T> {
    return (!ZERO && x >= xs && x < xe && row_ok) ? ur[(size_t)x * 64] : cmk<T>(0, 0);
  };
  // chunk q: output nodes xs + 5q - 4 + j (j < 5), rows y0 .. y0 + 3, entries [e]
  auto fetch_g = [&](int q) {
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      const int j = idx % CH, e = (idx / CH) % E, row = idx / (CH * E);
      const int x = xs + CH * q - 4 + j, yy = y0 + row;
      gp[i] = (idx < GN && x >= xs && x < xe && yy < g.ny)
                  ? G[(size_t)e * Np + linp_b(g, x, yy, 0)]
                  : cmk<T>(0, 0);
    }
  };
  auto store_g = [&](int q) {
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      if (idx < GN) (&gch[q & 1][0][0][0])[idx] = gp[i];
    }
  };
  auto step = [&](int k, auto ph) {
    constexpr int PH = decltype(ph)::value;  // k % 5
    col[PH][wv][lane] = pa[PH];
    col[PH][wv + 4][lane] = pb[PH];
    if (k + CH < nstep) fetch_col(xs - 2 + k + CH, pa[PH], pb[PH]);
    lds_barrier_b();
    if (PH == 0) {
      const int q = k / CH;
      if (CH * (q + 1) < nstep) store_g(q + 1);
      if (CH * (q + 2) < nstep) fetch_g(q + 2);
    }
#pragma unroll
    for (int dy = 0; dy < 5; ++dy) w[dy][PH] = col[PH][wv + dy][lane];
    const cpx<T> uo = uf[PH];
    if (!ZERO) uf[PH] = fetch_u(xs + k + 1);  // the output of step k + 5
    if (k >= 4 && row_ok) {
      const cpx<T>* gq = &gch[(k / CH) & 1][wv][0][PH];
      cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int dx = bsm_off<2, FORM>(e, 0), dy = bsm_off<2, FORM>(e, 1);
        acc = cfma(gq[e * CH], w[dy + 2][(PH + dx + 3) % 5], acc);
      }
      ur[(size_t)(xs + k - 4) * 64] = ZERO ? acc : (uo + acc);
    }
  };
  // prologue: columns of steps 0..4, u of their outputs, entries of chunks 0 (in LDS)
  // and 1 (in registers)
#pragma unroll
  for (int p = 0; p < CH; ++p) {
    fetch_col(xs - 2 + p, pa[p], pb[p]);
    uf[p] = fetch_u(xs + p - 4);
  }
  fetch_g(0);
  store_g(0);
  fetch_g(1);
#pragma unroll 1
  for (int k0 = 0; k0 < nstep; k0 += CH) {
    step(k0, std::integral_constant<int, 0>{});
    if (k0 + 1 < nstep) step(k0 + 1, std::integral_constant<int, 1>{});
    if (k0 + 2 < nstep) step(k0 + 2, std::integral_constant<int, 2>{});
    if (k0 + 3 < nstep) step(k0 + 3, std::integral_constant<int, 3>{});
    if (k0 + 4 < nstep) step(k0 + 4, std::integral_constant<int, 4>{});
  }
}

template <int FORM, class T>
static void launch_s64(Grid g, const void* G, const void* r, void* u, bool zero, hipStream_t st) {
  // balanced strips of at most B64_TX columns
  const int nsx = (g.nx + B64_TX - 1) / B64_TX;
  const int tx = (g.nx + nsx - 1) / nsx;
  const int nsx2 = (g.nx + tx - 1) / tx;
  const unsigned nb = (unsigned)nsx2 * (unsigned)((g.ny + B64_ROWS - 1) / B64_ROWS);
  if (zero)
    kb_sweep2d_s64<FORM, true, T><<<nb, 256, 0, st>>>(g, tx, (const cpx<T>*)G, (const cpx<T>*)r,
                                                      (cpx<T>*)u);
  else
    kb_sweep2d_s64<FORM, false, T><<<nb, 256, 0, st>>>(g, tx, (const cpx<T>*)G,
                                                       (const cpx<T>*)r, (cpx<T>*)u);
}

template <int FORM, class T, int P, bool LB = false>
static void launch_s64w(Grid g, int tx0, const void* G, const void* r, void* u, bool zero,
                        hipStream_t st) {
  static_assert(FORM == 2, "the walk relies on the zero entries of the assembled stencil");
  // balanced strips of at most tx0 columns; blocks of 4 rows (4 independent waves)
  const int nsx = (g.nx + tx0 - 1) / tx0;
  const int tx = (g.nx + nsx - 1) / nsx;
  const int nsx2 = (g.nx + tx - 1) / tx;
  const unsigned nb = (unsigned)nsx2 * (unsigned)((g.ny + 3) / 4);
  if (zero)
    kb_walk2d_s64<BOX2, OP_APPLY, T, T, T, P, true, LB><<<nb, 256, 0, st>>>(
        g, tx, (const cpx<T>*)G, (const cpx<T>*)r, nullptr, (cpx<T>*)u);
  else
    kb_walk2d_s64<BOX2, OP_ADD, T, T, T, P, true, LB><<<nb, 256, 0, st>>>(
        g, tx, (const cpx<T>*)G, (const cpx<T>*)r, nullptr, (cpx<T>*)u);
}

// 64-source 2D assembled sweep by tile code (S64_TILES candidates, 1-based): 1 = the LDS
// walk of four rows per block (16 columns per strip), 2..7 = the independent-wave walk
// with prefetch distance 2 or 3 over strips of 16, 32 or 64 columns, 8..10 = tiles 5..7
// with the smoother entries broadcast from LDS
template <int FORM, class T>
static void launch_s64_tile(int tile, Grid g, const void* G, const void* r, void* u, bool zero,
                            hipStream_t st) {
  static constexpr int TXS[3] = {16, 32, 64};
  if (tile == 0) tile = S64_DEFAULT_TILE;
  if (tile <= 1 || tile > S64_TILES) {
    launch_s64<FORM, T>(g, G, r, u, zero, st);
  } else if (tile <= 4) {
    launch_s64w<FORM, T, 2>(g, TXS[tile - 2], G, r, u, zero, st);
  } else if (tile <= 7) {
    launch_s64w<FORM, T, 3>(g, TXS[tile - 5], G, r, u, zero, st);
  } else {
    launch_s64w<FORM, T, 3, true>(g, TXS[tile - 8], G, r, u, zero, st);
  }
}

template <int FORM, class T, int LS>
static void launch_wide(Grid g, const void* G, const void* r, void* u, bool zero, size_t lds,
                        hipStream_t st) {
  const unsigned nb = (unsigned)(((g.nx + BW_NB - 1) / BW_NB) * g.ny);
  if (zero)
    kb_sweep2d_wide<FORM, true, T, LS><<<nb, 256, lds, st>>>(g, (const cpx<T>*)G,
                                                             (const cpx<T>*)r, (cpx<T>*)u);
  else
    kb_sweep2d_wide<FORM, false, T, LS><<<nb, 256, lds, st>>>(g, (const cpx<T>*)G,
                                                              (const cpx<T>*)r, (cpx<T>*)u);
}

// 3D assembled smoother, 16 sources: a block of 256 threads covers an x-y tile of
// 256/S nodes x S sources and walks along z.  The residual planes of the tile with a halo
// of 2 pass through a 6-slot LDS ring (one new plane per step, its loads issued a step
// ahead), so a residual value is loaded about (TX+4)(TY+4)/(TX TY) times per sweep instead
// of once per neighbour; the 125 smoother entries of a node are read by its S lanes as
// broadcast loads.  One barrier per step: plane k is written to slot k % 6 before the
// barrier of step k and read by steps k .. k + 4; its next writer, step k + 6, runs after
// the barrier of step k + 5, which every reader of step k + 4 has passed.
template <int LS>
struct Tile3 {
  static constexpr int S = 1 << LS, NT = 256 >> LS;
  static constexpr int TX = LS == 4 ? 4 : 8, TY = NT / TX;
  static constexpr int PX = TX + 4, PY = TY + 4, PV = PX * PY * S, PPT = (PV + 255) / 256;
};
constexpr int Z3_STRIP = 32;

template <bool ZERO, class T, int LS>
__global__ __launch_bounds__(256) void kb_sweep3d_zw(Grid g, int zt, const cpx<T>* __restrict__ G,
                                                     const cpx<T>* __restrict__ r,
                                                     cpx<T>* __restrict__ u) {
  using TL = Tile3<LS>;
  constexpr int S = TL::S, TX = TL::TX, TY = TL::TY, PX = TL::PX, PY = TL::PY, PV = TL::PV,
                PPT = TL::PPT;
  constexpr int E = shape_K<3, BOX2>();
  __shared__ cpx<T> ring[6][PV];
  const int nbx = (g.nx + TX - 1) / TX, nby = (g.ny + TY - 1) / TY;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int bx = (int)(b % (unsigned)nbx), by = (int)((b / (unsigned)nbx) % (unsigned)nby);
  const int bz = (int)(b / (unsigned)(nbx * nby));
  const int x0 = bx * TX, y0 = by * TY, zs = bz * zt;
  const int ze = min(zs + zt, g.nz);
  const int s = threadIdx.x & (S - 1), j = threadIdx.x >> LS;
  const int jx = j % TX, jy = j / TX;
  const int x = x0 + jx, y = y0 + jy;
  const bool ok = x < g.nx && y < g.ny;
  const size_t Np = (size_t)g.Np;
  cpx<T> pv[PPT];
  auto fetch = [&](int z) {
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
      const int v = (int)threadIdx.x + 256 * c;
      const int n = v >> LS, sv = v & (S - 1);
      const int gx = x0 + n % PX - 2, gy = y0 + n / PX - 2;
      pv[c] = (v < PV && inside_b(g, gx, gy, z)) ? r[(size_t)lin_b(g, gx, gy, z) * S + sv]
                                                 : cmk<T>(0, 0);
    }
  };
  const int nstep = ze - zs + 4;  // step k loads plane zs - 2 + k, outputs plane zs + k - 4
  auto step = [&](int k, auto ph) {
    constexpr int PH = decltype(ph)::value;  // k % 6
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
      const int v = (int)threadIdx.x + 256 * c;
      if (v < PV) ring[PH][v] = pv[c];
    }
    if (k + 1 < nstep) fetch(zs - 1 + k);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    const int z = zs + k - 4;
    if (k >= 4 && ok) {
      const long long ip = linp_b(g, x, y, z);
      const size_t o = (size_t)lin_b(g, x, y, z) * S + s;
      cpx<T> uo = cmk<T>(0, 0);
      if (!ZERO) uo = u[o];
      cpx<T> acc = cmk<T>(0, 0);
      // one plane of 25 entries at a time keeps 25 loads in flight per thread (the
      // register budget of several resident blocks) instead of all 125
#pragma unroll 1
      for (int dz = -2; dz <= 2; ++dz) {
        const cpx<T>* rp = &ring[(PH + dz + 4) % 6][0];
        const cpx<T>* gp = G + (size_t)(dz + 2) * 25 * Np + ip;
#pragma unroll
        for (int e = 0; e < 25; ++e) {
          const int dx = e % 5 - 2, dy = e / 5 - 2;
          acc = cfma(gp[(size_t)e * Np], rp[((jy + 2 + dy) * PX + (jx + 2 + dx)) * S + s], acc);
        }
      }
      u[o] = ZERO ? acc : (uo + acc);
    }
  };
  fetch(zs - 2);
#pragma unroll 1
  for (int k0 = 0; k0 < nstep; k0 += 6) {
    step(k0, std::integral_constant<int, 0>{});
    if (k0 + 1 < nstep) step(k0 + 1, std::integral_constant<int, 1>{});
    if (k0 + 2 < nstep) step(k0 + 2, std::integral_constant<int, 2>{});
    if (k0 + 3 < nstep) step(k0 + 3, std::integral_constant<int, 3>{});
    if (k0 + 4 < nstep) step(k0 + 4, std::integral_constant<int, 4>{});
    if (k0 + 5 < nstep) step(k0 + 5, std::integral_constant<int, 5>{});
  }
}

template <class T, int LS>
static void launch_zw(Grid g, const void* G, const void* r, void* u, bool zero, hipStream_t st) {
  using TL = Tile3<LS>;
  const int nsz = (g.nz + Z3_STRIP - 1) / Z3_STRIP;
  const int zt = (g.nz + nsz - 1) / nsz;
  const int nsz2 = (g.nz + zt - 1) / zt;
  const unsigned nb = (unsigned)(((g.nx + TL::TX - 1) / TL::TX) * ((g.ny + TL::TY - 1) / TL::TY) * nsz2);
  if (zero)
    kb_sweep3d_zw<true, T, LS><<<nb, 256, 0, st>>>(g, zt, (const cpx<T>*)G, (const cpx<T>*)r,
                                                   (cpx<T>*)u);
  else
    kb_sweep3d_zw<false, T, LS><<<nb, 256, 0, st>>>(g, zt, (const cpx<T>*)G, (const cpx<T>*)r,
                                                    (cpx<T>*)u);
}

template <int DIM, int FORM, class T>
static hipError_t bsweep_t(Grid g, int ls, int tile, const void* G, const void* r, void* u,
                           bool zero, hipStream_t st) {
  if constexpr (DIM == 3 && FORM == 2) {
    // measured: the z walk pays off with 16 sources; with fewer, the per-thread gather
    // through the caches below is faster
    if (ls == 4) {
      launch_zw<T, 4>(g, G, r, u, zero, st);
      VHB_CHECK();
      return hipSuccess;
    }
  }
  if constexpr (DIM == 2 && FORM == 2) {
    if (ls == 6) {
      launch_s64_tile<FORM, T>(tile, g, G, r, u, zero, st);
      VHB_CHECK();
      return hipSuccess;
    }
  }
  if (DIM == 2 && ls >= 4) {
    const size_t lds = ((size_t)bsm_entries<2, FORM>() * BW_NB +
                        (size_t)(BW_NB + 4) * 5 * ((size_t)1 << ls)) * sizeof(cpx<T>);
    if (lds <= 65536) {
      if (ls == 4)
        launch_wide<FORM, T, 4>(g, G, r, u, zero, lds, st);
      else if (ls == 5)
        launch_wide<FORM, T, 5>(g, G, r, u, zero, lds, st);
      else
        launch_wide<FORM, T, 6>(g, G, r, u, zero, lds, st);
      VHB_CHECK();
      return hipSuccess;
    }
  }
  if (DIM == 2) {
    const int NB = 256 >> ls;
    const unsigned nb = (unsigned)(((g.nx + NB - 1) / NB) * g.ny);
    const size_t lds = (size_t)(NB + 4) * 5 * ((size_t)1 << ls) * sizeof(cpx<T>);
    auto Gp = (const cpx<T>*)G;
    auto rp = (const cpx<T>*)r;
    auto up = (cpx<T>*)u;
    if (zero)
      kb_sweep2d<FORM, true, T><<<nb, 256, lds, st>>>(g, ls, Gp, rp, up);
    else
      kb_sweep2d<FORM, false, T><<<nb, 256, lds, st>>>(g, ls, Gp, rp, up);
    VHB_CHECK();
    return hipSuccess;
  }
  const unsigned nb = nblk(g.N << ls, 256);
  if (zero)
    kb_sweep<DIM, FORM, true, T><<<nb, 256, 0, st>>>(g, ls, (const cpx<T>*)G, (const cpx<T>*)r,
                                                     (cpx<T>*)u);
  else
    kb_sweep<DIM, FORM, false, T><<<nb, 256, 0, st>>>(g, ls, (const cpx<T>*)G, (const cpx<T>*)r,
                                                      (cpx<T>*)u);
  VHB_CHECK();
  return hipSuccess;
}

hipError_t batch_sweep(int dim, int form, Grid g, int ls, int prec, const void* G, const void* r,
                       void* u, bool zero, hipStream_t st, int tile) {
#define VHB_SW(D, F)                                                                \
  if (dim == D && form == F)                                                        \
    return prec == PREC_F64 ? bsweep_t<D, F, double>(g, ls, tile, G, r, u, zero, st) \
                            : bsweep_t<D, F, float>(g, ls, tile, G, r, u, zero, st);
  VHB_SW(2, 0) VHB_SW(3, 0) VHB_SW(2, 1) VHB_SW(3, 1) VHB_SW(2, 2) VHB_SW(3, 2)
  VHB_SW(2, 3) VHB_SW(3, 3) VHB_SW(2, 4) VHB_SW(3, 4) VHB_SW(2, 5) VHB_SW(3, 5)
#undef VHB_SW
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ transfers, batched
template <int DIM, int RF, class T>
__global__ __launch_bounds__(256) void kb_restrict(Grid gf, Grid gc, int ls,
                                                   const cpx<T>* __restrict__ r,
                                                   cpx<T>* __restrict__ rc) {
  unsigned I;
  int s;
  if (!thread_ns(gc, ls, I, s)) return;
  int Ix, Iy, Iz;
  decode_b(I, gc, Ix, Iy, Iz);
  const int S = 1 << ls;
  constexpr int RR = fam_radius(RF), RW = 2 * RR + 1, NT = ipow(RW, DIM);
  cpx<T> acc = cmk<T>(0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int tx = t % RW - RR, ty = (t / RW) % RW - RR, tz = (DIM == 3) ? t / (RW * RW) - RR : 0;
    const int fx = 2 * Ix + tx, fy = 2 * Iy + ty, fz = 2 * Iz + tz;
    if (inside_b(gf, fx, fy, fz)) {
      const T w = (T)(fam_r(RF, tx) * fam_r(RF, ty) * (DIM == 3 ? fam_r(RF, tz) : 1.0));
      acc = cfma(cmk<T>(w, 0), r[(size_t)lin_b(gf, fx, fy, fz) * S + s], acc);
    }
  }
  rc[(size_t)I * S + s] = acc;
}

template <int DIM, int PF, class T>
__global__ __launch_bounds__(256) void kb_prolong_add(Grid gf, Grid gc, int ls,
                                                      const cpx<T>* __restrict__ e,
                                                      cpx<T>* __restrict__ u) {
  unsigned i;
  int s;
  if (!thread_ns(gf, ls, i, s)) return;
  int c[3];
  decode_b(i, gf, c[0], c[1], c[2]);
  const int S = 1 << ls;
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
        if (wt != (T)0 && inside_b(gc, Jx, Jy, Jz))
          acc = cfma(cmk<T>(wt, 0), e[(size_t)lin_b(gc, Jx, Jy, Jz) * S + s], acc);
      }
  const size_t o = (size_t)i * S + s;
  u[o] = u[o] + acc;
}

hipError_t batch_restrict(int dim, int rf, Grid gf, Grid gc, int ls, int prec, const void* r,
                          void* rc, hipStream_t st) {
  const unsigned nb = nblk(gc.N << ls, 256);
#define VHB_RS(D, R, T)                                                                          \
  if (dim == D && rf == R) {                                                                     \
    kb_restrict<D, R, T><<<nb, 256, 0, st>>>(gf, gc, ls, (const cpx<T>*)r, (cpx<T>*)rc);          \
    VHB_CHECK();                                                                                 \
    return hipSuccess;                                                                           \
  }
  if (prec == PREC_F64) {
    VHB_RS(2, FAM_LINEAR, double) VHB_RS(2, FAM_CUBIC, double)
    VHB_RS(3, FAM_LINEAR, double) VHB_RS(3, FAM_CUBIC, double)
  } else {
    VHB_RS(2, FAM_LINEAR, float) VHB_RS(2, FAM_CUBIC, float)
    VHB_RS(3, FAM_LINEAR, float) VHB_RS(3, FAM_CUBIC, float)
  }
#undef VHB_RS
  return hipErrorInvalidValue;
}

hipError_t batch_prolong_add(int dim, int pf, Grid gf, Grid gc, int ls, int prec, const void* e,
                             void* u, hipStream_t st) {
  const unsigned nb = nblk(gf.N << ls, 256);
#define VHB_PA(D, P, T)                                                                          \
  if (dim == D && pf == P) {                                                                     \
    kb_prolong_add<D, P, T><<<nb, 256, 0, st>>>(gf, gc, ls, (const cpx<T>*)e, (cpx<T>*)u);        \
    VHB_CHECK();                                                                                 \
    return hipSuccess;                                                                           \
  }
  if (prec == PREC_F64) {
    VHB_PA(2, FAM_LINEAR, double) VHB_PA(2, FAM_CUBIC, double)
    VHB_PA(3, FAM_LINEAR, double) VHB_PA(3, FAM_CUBIC, double)
  } else {
    VHB_PA(2, FAM_LINEAR, float) VHB_PA(2, FAM_CUBIC, float)
    VHB_PA(3, FAM_LINEAR, float) VHB_PA(3, FAM_CUBIC, float)
  }
#undef VHB_PA
  return hipErrorInvalidValue;
}

// Y[row][s] = sum_j D[row][j] X[j][s], D the FP64 coarsest inverse (one thread per (row, s))
// Y = D X for the coarsest level (D the dense FP64 inverse, n x n; X, Y n x S): each
// output is summed by DKS threads over interleaved columns, then combined in LDS in a
// fixed order, so that the short coarsest solve spreads over enough blocks
constexpr int DKS = 8;

template <class T>
__global__ __launch_bounds__(256) void kb_dense(int n, int ls, const cpx<double>* __restrict__ D,
                                                const cpx<T>* __restrict__ X,
                                                cpx<T>* __restrict__ Y) {
  __shared__ cpx<double> red[DKS][256 / DKS];
  constexpr int OB = 256 / DKS;  // outputs per block
  const int ks = threadIdx.x / OB, ob = threadIdx.x % OB;
  const long long t = (long long)blockIdx.x * OB + ob;  // output (row, source)
  const bool valid = t < ((long long)n << ls);
  const int row = valid ? (int)(t >> ls) : 0, s = (int)(t & ((1 << ls) - 1));
  const int S = 1 << ls;
  cpx<double> acc = cmk(0.0, 0.0);
  if (valid)
    for (int j = ks; j < n; j += DKS)
      acc = cfma(D[(size_t)row * n + j], ccast<double>(X[(size_t)j * S + s]), acc);
  red[ks][ob] = acc;
  __syncthreads();
  if (ks == 0 && valid) {
    cpx<double> sum = red[0][ob];
    for (int k = 1; k < DKS; ++k) sum = sum + red[k][ob];
    Y[t] = ccast<T>(sum);
  }
}

hipError_t batch_dense(int n, int ls, const cpx<double>* D, int prec, const void* X, void* Y,
                       hipStream_t st) {
  const unsigned nb = nblk((long long)n << ls, 256 / DKS);
  if (prec == PREC_F64)
    kb_dense<double><<<nb, 256, 0, st>>>(n, ls, D, (const cpx<double>*)X, (cpx<double>*)Y);
  else
    kb_dense<float><<<nb, 256, 0, st>>>(n, ls, D, (const cpx<float>*)X, (cpx<float>*)Y);
  VHB_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------ Krylov, batched (FP64)
// Block-partial per-source multi-dots over a contiguous chunk of nodes:
//   mode 0: part[b][j][s] = sum_i conj(V_j[i][s]) w[i][s]
//   mode 1: w -= sum_j h[j][s] V_j, then the same dots with the updated w
//   mode 2: w -= sum_j h[j][s] V_j, part[b][0][s] = ||w[., s]||^2
constexpr int BKMAX = 65;

template <int MODE>
__global__ __launch_bounds__(256) void kb_cgs(const cpx<double>* __restrict__ V, size_t ldv, int nv,
                                              const cpx<double>* __restrict__ h,
                                              cpx<double>* __restrict__ w, long long N, int ls,
                                              cpx<double>* __restrict__ part) {
  __shared__ cpx<double> red[4][64];
  const int S = 1 << ls;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = lane & (S - 1);
  const int nodes_per_block = 256 >> ls;
  const int sub = threadIdx.x >> ls;  // node slot within the block
  const long long per = (N + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < N ? lo + per : N;
  const int nout = (MODE == 2) ? 1 : nv;
  for (int j0 = 0; j0 < nout; j0 += 8) {
    cpx<double> acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = cmk(0.0, 0.0);
    for (long long i = lo + sub; i < hi; i += nodes_per_block) {
      const size_t o = (size_t)i * S + s;
      cpx<double> wi = w[o];
      if (MODE != 0 && j0 == 0) {
        for (int j = 0; j < nv; ++j) wi = wi - h[(size_t)j * 64 + s] * V[(size_t)j * ldv + o];
        w[o] = wi;
      }
      if (MODE == 2) {
        acc[0].re += wi.re * wi.re + wi.im * wi.im;
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (j0 + q < nv) acc[q] = cfma_conj(V[(size_t)(j0 + q) * ldv + o], wi, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (j0 + q >= nout) break;
      cpx<double> v = acc[q];
      // lanes with the same source: stride S within the wavefront
      for (int o = 32; o >= S; o >>= 1) {
        v.re += __shfl_down(v.re, o, 64);
        v.im += __shfl_down(v.im, o, 64);
      }
      __syncthreads();
      if (lane < S) red[wv][lane] = v;
      __syncthreads();
      if (threadIdx.x < S) {
        cpx<double> t = red[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) t = t + red[k][threadIdx.x];
        part[((size_t)blockIdx.x * BKMAX + j0 + q) * 64 + threadIdx.x] = t;
      }
    }
    if (MODE != 0) __syncthreads();
  }
}

// Register-resident form of kb_cgs for nv <= NJ: one sweep over the nodes does the
// whole pass.  Each thread keeps one accumulator per basis vector; in MODE 1 the
// update and the new dot products read V[j] at the same node back to back, so the
// second read hits the cache and V leaves HBM once per pass.  w is read once.
template <int MODE, int NJ>
__global__ __launch_bounds__(256) void kb_cgs_r(const cpx<double>* __restrict__ V, size_t ldv,
                                                int nv, const cpx<double>* __restrict__ h,
                                                cpx<double>* __restrict__ w, long long N, int ls,
                                                cpx<double>* __restrict__ part) {
  constexpr int NA = (MODE == 2) ? 1 : NJ;
  __shared__ cpx<double> hs[MODE == 0 ? 1 : NJ][64];
  __shared__ cpx<double> red[4][64];
  const int S = 1 << ls;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = lane & (S - 1);
  if (MODE != 0) {
    for (int e = threadIdx.x; e < NJ * 64; e += 256)
      hs[e >> 6][e & 63] = (e >> 6) < nv ? h[e] : cmk(0.0, 0.0);
    __syncthreads();
  }
  // Nodes are dealt to the blocks round-robin, a row of nodes_per_block at a time, so
  // that at any moment the whole grid reads one narrow window of every column.
  const int nodes_per_block = 256 >> ls;
  const int sub = threadIdx.x >> ls;
  const long long stride = (long long)gridDim.x * nodes_per_block;
  cpx<double> acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = cmk(0.0, 0.0);
  // Columns j >= nv re-read column nv - 1 (a cache hit) with a zero coefficient, and
  // their sums are discarded: every load is unconditional, so all of a node's loads
  // are in flight together.
  for (long long i = (long long)blockIdx.x * nodes_per_block + sub; i < N; i += stride) {
    const size_t o = (size_t)i * S + s;
    cpx<double> wi = w[o];
    if (MODE != 0 && nv > 0) {  // the norm-only pass at a restart has nv == 0
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        wi = wi - hs[j][s] * V[(size_t)(j < nv ? j : nv - 1) * ldv + o];
      w[o] = wi;
    }
    if (MODE == 2) {
      acc[0].re += wi.re * wi.re + wi.im * wi.im;
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc[j] = cfma_conj(V[(size_t)(j < nv ? j : nv - 1) * ldv + o], wi, acc[j]);
    }
  }
  const int nout = (MODE == 2) ? 1 : nv;
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    if (q < nout) {  // nout is uniform over the block
      cpx<double> v = acc[q];
      for (int k = 32; k >= S; k >>= 1) {
        v.re += __shfl_down(v.re, k, 64);
        v.im += __shfl_down(v.im, k, 64);
      }
      __syncthreads();
      if (lane < S) red[wv][lane] = v;
      __syncthreads();
      if (threadIdx.x < S) {
        cpx<double> t = red[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) t = t + red[k][threadIdx.x];
        part[((size_t)blockIdx.x * BKMAX + q) * 64 + threadIdx.x] = t;
      }
    }
  }
}

// Two-level fixed-order reduction of the partial sums, out[j][s] = sum_b part[b][j][s].
// Level 1: block (j, slice) sums the rows b = slice, slice + RSL, ... (256/S row
// groups x S sources, then a tree over the groups); level 2 sums the RSL slices.
constexpr int RSL = 16;

__global__ __launch_bounds__(256) void kb_reduce(const cpx<double>* __restrict__ part, int nb,
                                                 int ls, cpx<double>* __restrict__ part2) {
  __shared__ cpx<double> sh[256];
  const int S = 1 << ls;
  const int j = blockIdx.x, sl = blockIdx.y, t = threadIdx.x;
  const int s = t & (S - 1), grp = t >> ls, ngrp = 256 >> ls;
  cpx<double> acc = cmk(0.0, 0.0);
  for (int b = sl + RSL * grp; b < nb; b += RSL * ngrp)
    acc = acc + part[((size_t)b * BKMAX + j) * 64 + s];
  sh[t] = acc;
  __syncthreads();
  for (int w = 128; w >= S; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  if (t < S) part2[((size_t)j * RSL + sl) * 64 + t] = sh[t];
}

__global__ void kb_reduce_fin(const cpx<double>* __restrict__ part2, int S,
                              cpx<double>* __restrict__ out) {
  const int j = blockIdx.x, s = threadIdx.x;
  if (s >= S) return;
  cpx<double> acc = cmk(0.0, 0.0);
  for (int sl = 0; sl < RSL; ++sl) acc = acc + part2[((size_t)j * RSL + sl) * 64 + s];
  out[(size_t)j * 64 + s] = acc;
}

// Blocks of 256 threads that are resident at once on the whole device for kernel k
// (queried once per kernel; every device the library runs on is the same gfx950 part).
template <class K>
static int resident_blocks(K k) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 256, 0) != hipSuccess || per < 1)
    return 1 << 30;
  return per * ncu;
}

// one pass with a grid of exactly one resident wave of blocks (a partial second wave
// would leave most of the device idle at the end); returns the number of partial rows
template <int MODE, int NJ>
static int cgs_r(const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h, cpx<double>* w,
                 long long N, int ls, cpx<double>* part, int nb, hipStream_t st) {
  static const int res = resident_blocks(kb_cgs_r<MODE, NJ>);
  const int g = nb < res ? nb : res;
  kb_cgs_r<MODE, NJ><<<g, 256, 0, st>>>(V, ldv, nv, h, w, N, ls, part);
  return g;
}

template <int MODE>
static int cgs_launch(const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                      cpx<double>* w, long long N, int ls, cpx<double>* part, int nb,
                      hipStream_t st) {
  if (nv <= 8) return cgs_r<MODE, 8>(V, ldv, nv, h, w, N, ls, part, nb, st);
  if (nv <= 16) return cgs_r<MODE, 16>(V, ldv, nv, h, w, N, ls, part, nb, st);
  if (nv <= 24) return cgs_r<MODE, 24>(V, ldv, nv, h, w, N, ls, part, nb, st);
  kb_cgs<MODE><<<nb, 256, 0, st>>>(V, ldv, nv, h, w, N, ls, part);
  return nb;
}

hipError_t batch_cgs(int mode, const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                     cpx<double>* w, long long N, int ls, cpx<double>* part, int nb,
                     cpx<double>* out, hipStream_t st) {
  if (nv < (mode == 2 ? 0 : 1) || nv > BKMAX) return hipErrorInvalidValue;
  int rows;
  if (mode == 0)
    rows = cgs_launch<0>(V, ldv, nv, h, w, N, ls, part, nb, st);
  else if (mode == 1)
    rows = cgs_launch<1>(V, ldv, nv, h, w, N, ls, part, nb, st);
  else
    rows = cgs_launch<2>(V, ldv, nv, h, w, N, ls, part, nb, st);
  VHB_CHECK();
  // the slice sums live after the nb partial rows (the workspace holds both)
  cpx<double>* part2 = part + (size_t)nb * BKMAX * 64;
  const int nout = mode == 2 ? 1 : nv;
  kb_reduce<<<dim3(nout, RSL), 256, 0, st>>>(part, rows, ls, part2);
  VHB_CHECK();
  kb_reduce_fin<<<nout, 64, 0, st>>>(part2, 1 << ls, out);
  VHB_CHECK();
  return hipSuccess;
}

// Arnoldi column j for every source (one thread per source): same algebra as the
// single-source kernel, on the per-source arrays of BatchKrylovDev.
__global__ void kb_finalize(BatchKrylovDev* __restrict__ K, int j, int S) {
  const int s = threadIdx.x;
  if (s >= S) return;
  const int ldh = MMAX + 1;
  auto H = [&](int col, int row) -> cpx<double>& {
    return K->H[((size_t)col * ldh + row) * 64 + s];
  };
#pragma unroll 8
  for (int i = 0; i <= j; ++i) H(j, i) = K->h1[i * 64 + s] + K->h2[i * 64 + s];
  const double nrm = sqrt(K->nrm2[s].re);
  H(j, j + 1) = cmk(nrm, 0.0);
#pragma unroll 8
  for (int i = 0; i < j; ++i) {
    const cpx<double> a = H(j, i), b = H(j, i + 1);
    const double c = K->cs[i * 64 + s];
    const cpx<double> sn = K->sn[i * 64 + s];
    H(j, i) = c * a + sn * b;
    H(j, i + 1) = c * b - cmk(sn.re, -sn.im) * a;
  }
  const cpx<double> a = H(j, j);
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
    sn = cmk(a.re / aa * b / r, a.im / aa * b / r);
  }
  K->cs[j * 64 + s] = c;
  K->sn[j * 64 + s] = sn;
  H(j, j) = c * a + sn * cmk(b, 0.0);
  H(j, j + 1) = cmk(0.0, 0.0);
  const cpx<double> gj = K->g[j * 64 + s];
  K->g[(j + 1) * 64 + s] = cmk(0.0, 0.0) - cmk(sn.re, -sn.im) * gj;
  K->g[j * 64 + s] = c * gj;
  const cpx<double> gn = K->g[(j + 1) * 64 + s];
  const double est = sqrt(gn.re * gn.re + gn.im * gn.im);
  K->status[s * 4 + 0] = est;
  K->status[s * 4 + 1] = nrm;
  K->inv_nrm[s] = (nrm > 0.0) ? 1.0 / nrm : 0.0;
  K->status[s * 4 + 2] = (!(nrm == nrm) || !(est == est) || isinf(nrm)) ? 1.0 : 0.0;
}

__global__ void kb_cycle_init(BatchKrylovDev* __restrict__ K, int m, int S) {
  const int s = threadIdx.x;
  if (s >= S) return;
  const double beta = sqrt(K->nrm2[s].re);
  K->g[s] = cmk(beta, 0.0);
  for (int i = 1; i <= m; ++i) K->g[i * 64 + s] = cmk(0.0, 0.0);
  K->inv_nrm[s] = beta > 0.0 ? 1.0 / beta : 0.0;
  K->status[s * 4 + 3] = beta;
}

// y = R^{-1} g over the first kcols[s] columns of source s (0: nothing to update)
// the solved y_q are kept in LDS as they are produced, so that the inner products read
// only H from memory (loads independent of each other, issued several at a time)
__global__ void kb_backsolve(BatchKrylovDev* __restrict__ K, int S) {
  __shared__ cpx<double> ys[MMAX][64];
  const int s = threadIdx.x;
  if (s >= S) return;
  const int ldh = MMAX + 1;
  const int k = K->kcols[s];
  for (int i = k - 1; i >= 0; --i) {
    cpx<double> acc = K->g[i * 64 + s];
#pragma unroll 8
    for (int q = i + 1; q < k; ++q)
      acc = acc - K->H[((size_t)q * ldh + i) * 64 + s] * ys[q][s];
    const cpx<double> yi = acc * cinv(K->H[((size_t)i * ldh + i) * 64 + s]);
    ys[i][s] = yi;
    K->y[i * 64 + s] = yi;
  }
}

// x[i][s] += sum_{j < kcols[s]} y[j][s] Z_j[i][s]
template <class TZ>
__global__ __launch_bounds__(256) void kb_update_x(const BatchKrylovDev* __restrict__ K, int kmax,
                                                   const cpx<TZ>* __restrict__ Z, size_t ldz,
                                                   cpx<double>* __restrict__ x, long long N,
                                                   int ls) {
  const long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= (N << ls)) return;
  const int s = (int)(t & ((1 << ls) - 1));
  const int k = K->kcols[s];
  cpx<double> a = x[t];
  for (int j = 0; j < kmax; ++j)
    if (j < k) a = cfma(K->y[j * 64 + s], ccast<double>(Z[(size_t)j * ldz + t]), a);
  x[t] = a;
}

// v[i][s] = w[i][s] * inv_nrm[s]
__global__ __launch_bounds__(256) void kb_scale(const BatchKrylovDev* __restrict__ K,
                                                const cpx<double>* __restrict__ w,
                                                cpx<double>* __restrict__ v, long long N, int ls) {
  const long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= (N << ls)) return;
  v[t] = K->inv_nrm[t & ((1 << ls) - 1)] * w[t];
}

// ------------------------------------------------------------------ delayed CGS2
// Delayed classical Gram-Schmidt with one reorthogonalisation (the reorthogonalisation
// of each basis vector is merged into the next step's projection).  At step j the
// basis holds final columns v_0..v_{j-1}, the lagged vector u = V_j (projected once,
// scaled to about unit norm) and w = A z_j, z_j = M^{-1} u.  Pass A (one read of the
// basis) gives b = V^H u, d = V^H w, u^H w, u^H u, w^H w; then
//   v_j = (u - V b) / beta,  beta^2 = u^H u - |b|^2,
//   A z_{j-1} = V (c' + nu' b) + nu' beta v_j     (Hessenberg column j-1 completed),
//   c = [d; (u^H w - b^H d) / beta] = the first projection of w on v_0..v_j,
//   u' = (w - V d' - gam u) / nu, d' = d - b c_j / beta, gam = c_j / beta,
//   nu^2 = w^H w - |c|^2,
// and pass B (a second read) writes v_j and u'.  FGMRES accepts z_j = M^{-1} u in place
// of M^{-1} v_j because it keeps Z: A Z = V H holds column by column.

// pass A over the columns [c0, c0 + nc) of one group; the first group also sums the
// three products of u and w.  Output rows: b (nc), d (nc), then u^H w, u^H u, w^H w.
template <int NJ>
__global__ __launch_bounds__(256) void kb_dcgs_a(const cpx<double>* __restrict__ V, size_t ldv,
                                                 int c0, int nc, int j, int wcol, int first,
                                                 long long N, int ls,
                                                 cpx<double>* __restrict__ part) {
  __shared__ cpx<double> red[4][64];
  const int S = 1 << ls;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = lane & (S - 1);
  const int nodes_per_block = 256 >> ls;
  const int sub = threadIdx.x >> ls;
  const long long stride = (long long)gridDim.x * nodes_per_block;
  const cpx<double>* u = V + (size_t)j * ldv;
  const cpx<double>* w = V + (size_t)wcol * ldv;
  cpx<double> ab[NJ], ad[NJ], e = cmk(0.0, 0.0), f = cmk(0.0, 0.0), gw = cmk(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < NJ; ++q) ab[q] = ad[q] = cmk(0.0, 0.0);
  for (long long i = (long long)blockIdx.x * nodes_per_block + sub; i < N; i += stride) {
    const size_t o = (size_t)i * S + s;
    const cpx<double> ui = u[o], wi = w[o];
    if (nc > 0) {
#pragma unroll
      for (int q = 0; q < NJ; ++q) {
        const cpx<double> v = V[(size_t)(c0 + (q < nc ? q : nc - 1)) * ldv + o];
        ab[q] = cfma_conj(v, ui, ab[q]);
        ad[q] = cfma_conj(v, wi, ad[q]);
      }
    }
    if (first) {
      e = cfma_conj(ui, wi, e);
      f.re += ui.re * ui.re + ui.im * ui.im;
      gw.re += wi.re * wi.re + wi.im * wi.im;
    }
  }
  // rows in the layout of K->pa: b at [0, DG), d at [DG, 2 DG), then u^H w, u^H u, w^H w
  // (rows past nc hold sums that are never read)
#pragma unroll
  for (int q = 0; q < 2 * DG + 3; ++q) {
    cpx<double> v = cmk(0.0, 0.0);
    if (q < DG) {
      if (q < NJ) v = ab[q < NJ ? q : 0];
    } else if (q < 2 * DG) {
      if (q - DG < NJ) v = ad[q - DG < NJ ? q - DG : 0];
    } else {
      v = q == 2 * DG ? e : (q == 2 * DG + 1 ? f : gw);
    }
    for (int k = 32; k >= S; k >>= 1) {
      v.re += __shfl_down(v.re, k, 64);
      v.im += __shfl_down(v.im, k, 64);
    }
    __syncthreads();
    if (lane < S) red[wv][lane] = v;
    __syncthreads();
    if (threadIdx.x < S) {
      cpx<double> t = red[0][threadIdx.x];
      for (int k = 1; k < 4; ++k) t = t + red[k][threadIdx.x];
      part[((size_t)blockIdx.x * BKMAX + q) * 64 + threadIdx.x] = t;
    }
  }
}

template <int NJ>
static int dcgs_a_launch(const cpx<double>* V, size_t ldv, int c0, int nc, int j, int wcol,
                         int first, long long N, int ls, cpx<double>* part, int nb,
                         hipStream_t st) {
  static const int res = resident_blocks(kb_dcgs_a<NJ>);
  const int g = nb < res ? nb : res;
  kb_dcgs_a<NJ><<<g, 256, 0, st>>>(V, ldv, c0, nc, j, wcol, first, N, ls, part);
  return g;
}

hipError_t batch_dcgs_a(const cpx<double>* V, size_t ldv, int j, int wcol, long long N, int ls,
                        cpx<double>* part, int nb, BatchKrylovDev* K, hipStream_t st) {
  if (j < 0 || j > MMAX || wcol < j || wcol > MMAX) return hipErrorInvalidValue;
  const int ng = j > 0 ? (j + DG - 1) / DG : 1;
  cpx<double>* part2 = part + (size_t)nb * BKMAX * 64;
  for (int q = 0; q < ng; ++q) {
    const int c0 = q * DG, nc = j - c0 < DG ? j - c0 : DG;
    const int first = q == 0;
    int rows;
    if (nc <= 4)
      rows = dcgs_a_launch<4>(V, ldv, c0, nc, j, wcol, first, N, ls, part, nb, st);
    else if (nc <= 8)
      rows = dcgs_a_launch<8>(V, ldv, c0, nc, j, wcol, first, N, ls, part, nb, st);
    else
      rows = dcgs_a_launch<DG>(V, ldv, c0, nc, j, wcol, first, N, ls, part, nb, st);
    VHB_CHECK();
    kb_reduce<<<dim3(PA_ROWS, RSL), 256, 0, st>>>(part, rows, ls, part2);
    VHB_CHECK();
    kb_reduce_fin<<<PA_ROWS, 64, 0, st>>>(part2, 1 << ls, K->pa + (size_t)q * PA_ROWS * 64);
    VHB_CHECK();
  }
  return hipSuccess;
}

// one thread per source: complete Hessenberg column j-1 (j >= 1) with its Givens
// rotation and residual estimate; unless closing, prepare pass B of step j
__global__ void kb_dcgs_fin(BatchKrylovDev* __restrict__ K, int j, int S, int closing) {
  const int s = threadIdx.x;
  if (s >= S) return;
  const int ldh = MMAX + 1;
  auto H = [&](int col, int row) -> cpx<double>& {
    return K->H[((size_t)col * ldh + row) * 64 + s];
  };
  auto bv = [&](int i) {
    const int q = i / DG, li = i % DG;
    return K->pa[((size_t)q * PA_ROWS + li) * 64 + s];
  };
  auto dv = [&](int i) {
    const int q = i / DG, li = i % DG;
    return K->pa[((size_t)q * PA_ROWS + DG + li) * 64 + s];
  };
  const cpx<double> e = K->pa[(size_t)(2 * DG) * 64 + s];
  const double f = K->pa[(size_t)(2 * DG + 1) * 64 + s].re;
  const double gw = K->pa[(size_t)(2 * DG + 2) * 64 + s].re;
  double beta = 1.0;
  bool bad = false;
  if (j >= 1) {
    double bb = 0.0;
#pragma unroll 8
    for (int i = 0; i < j; ++i) {
      const cpx<double> b = bv(i);
      bb += b.re * b.re + b.im * b.im;
    }
    const double b2 = f - bb;
    beta = b2 > 0.0 ? sqrt(b2) : 0.0;
    const double nu = K->nuprev[s];
    const int jj = j - 1;  // the column completed now
#pragma unroll 8
    for (int i = 0; i < j; ++i) H(jj, i) = K->cprev[i * 64 + s] + nu * bv(i);
    const double nrm = nu * beta;
#pragma unroll 8
    for (int i = 0; i < jj; ++i) {
      const cpx<double> a = H(jj, i), b = H(jj, i + 1);
      const double c = K->cs[i * 64 + s];
      const cpx<double> sn = K->sn[i * 64 + s];
      H(jj, i) = c * a + sn * b;
      H(jj, i + 1) = c * b - cmk(sn.re, -sn.im) * a;
    }
    const cpx<double> a = H(jj, jj);
    double c;
    cpx<double> sn;
    const double aa = sqrt(a.re * a.re + a.im * a.im);
    if (aa == 0.0) {
      c = 0.0;
      sn = cmk(1.0, 0.0);
    } else {
      const double r = sqrt(aa * aa + nrm * nrm);
      c = aa / r;
      sn = cmk(a.re / aa * nrm / r, a.im / aa * nrm / r);
    }
    K->cs[jj * 64 + s] = c;
    K->sn[jj * 64 + s] = sn;
    H(jj, jj) = c * a + sn * cmk(nrm, 0.0);
    H(jj, jj + 1) = cmk(0.0, 0.0);
    const cpx<double> gj = K->g[jj * 64 + s];
    K->g[(jj + 1) * 64 + s] = cmk(0.0, 0.0) - cmk(sn.re, -sn.im) * gj;
    K->g[jj * 64 + s] = c * gj;
    const cpx<double> gn = K->g[(jj + 1) * 64 + s];
    const double est = sqrt(gn.re * gn.re + gn.im * gn.im);
    K->status[s * 4 + 0] = est;
    K->status[s * 4 + 1] = nrm;
    bad = !(nrm == nrm) || !(est == est) || isinf(nrm);
  }
  if (!closing) {
    const double ibeta = beta > 0.0 ? 1.0 / beta : 0.0;
    cpx<double> bd = cmk(0.0, 0.0);
#pragma unroll 8
    for (int i = 0; i < j; ++i) {
      const cpx<double> b = bv(i);
      bd = cfma_conj(b, dv(i), bd);
    }
    const cpx<double> cj = ibeta * (e - bd);
    const cpx<double> gam = ibeta * cj;
    double cc = cj.re * cj.re + cj.im * cj.im;
#pragma unroll 8
    for (int i = 0; i < j; ++i) {
      const cpx<double> d = dv(i), b = bv(i);
      cc += d.re * d.re + d.im * d.im;
      K->cprev[i * 64 + s] = d;
      K->xb[i * 64 + s] = b;
      K->yd[i * 64 + s] = d - b * gam;
    }
    K->cprev[j * 64 + s] = cj;
    const double n2 = gw - cc;
    const double nu = n2 > 1e-28 * gw ? sqrt(n2) : sqrt(1e-28 * gw);
    K->nuprev[s] = nu;
    K->gam[s] = gam;
    K->ib[s] = ibeta;
    K->inu[s] = nu > 0.0 ? 1.0 / nu : 0.0;
    bad = bad || !(nu == nu) || isinf(nu) || !(cj.re == cj.re) || !(cj.im == cj.im);
  }
  K->status[s * 4 + 2] = bad ? 1.0 : 0.0;
}

// pass B over the column group [c0, c0 + nc): t0 = V_j - sum xb_i v_i,
// t1 = V_{j+1} - sum yd_i v_i (minus gam u in the first group); the last group scales
// by ib and inu.  Columns past nc re-read the last one with a zero coefficient.
// Pass B over columns c0 .. c0+nc-1 of the basis in one sweep of the vectors: the
// coefficients of every column and source sit in LDS ([column][source], nc * S each for
// x and y), the columns are taken eight at a time with their loads in flight together,
// and u, w are read and written once however many columns there are.
__global__ __launch_bounds__(256) void kb_dcgs_b(cpx<double>* __restrict__ V, size_t ldv, int c0,
                                                 int nc, int j, int first, int last, long long N,
                                                 int ls, const BatchKrylovDev* __restrict__ K,
                                                 cpx<float>* __restrict__ lo) {
  extern __shared__ cpx<double> cs[];
  const int S = 1 << ls;
  cpx<double>* xs = cs;
  cpx<double>* ys = cs + (size_t)nc * S;
  for (int e = threadIdx.x; e < nc * S; e += 256) {
    const int q = e >> ls, sv = e & (S - 1);
    xs[e] = K->xb[(size_t)(c0 + q) * 64 + sv];
    ys[e] = K->yd[(size_t)(c0 + q) * 64 + sv];
  }
  __syncthreads();
  const int s = threadIdx.x & (S - 1);
  const cpx<double> gam = K->gam[s];
  const double ib = K->ib[s], inu = K->inu[s];
  cpx<double>* u = V + (size_t)j * ldv;
  cpx<double>* w = V + (size_t)(j + 1) * ldv;
  const long long total = N << ls;
  constexpr int UN = 8;
  for (long long t = (long long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const size_t o = (size_t)t;
    cpx<double> t0 = u[o], t1 = w[o];
    if (first) t1 = t1 - gam * t0;
    int q = 0;
    for (; q + UN <= nc; q += UN) {
      cpx<double> v[UN];
#pragma unroll
      for (int r = 0; r < UN; ++r) v[r] = V[(size_t)(c0 + q + r) * ldv + o];
#pragma unroll
      for (int r = 0; r < UN; ++r) {
        t0 = t0 - xs[(q + r) * S + s] * v[r];
        t1 = t1 - ys[(q + r) * S + s] * v[r];
      }
    }
    for (; q < nc; ++q) {
      const cpx<double> v = V[(size_t)(c0 + q) * ldv + o];
      t0 = t0 - xs[q * S + s] * v;
      t1 = t1 - ys[q * S + s] * v;
    }
    if (last) {
      t0 = ib * t0;
      t1 = inu * t1;
      if (lo) lo[o] = ccast<float>(t1);
    }
    u[o] = t0;
    w[o] = t1;
  }
}

hipError_t batch_dcgs_fin(BatchKrylovDev* K, int j, int S, int closing, hipStream_t st) {
  if (j < 0 || j > MMAX) return hipErrorInvalidValue;
  kb_dcgs_fin<<<1, 64, 0, st>>>(K, j, S, closing);
  VHB_CHECK();
  return hipSuccess;
}

hipError_t batch_dcgs_b(cpx<double>* V, size_t ldv, int j, long long N, int ls,
                        const BatchKrylovDev* K, cpx<float>* lo, hipStream_t st) {
  if (j < 0 || j >= MMAX) return hipErrorInvalidValue;
  // columns per sweep: the coefficients of all of them in at most 48 KB of LDS (every
  // column in one sweep up to 24 columns at 64 sources, 48 at 32, ...)
  const int S = 1 << ls;
  const int gb = (48 * 1024) / (2 * S * (int)sizeof(cpx<double>));
  const int ng = j > 0 ? (j + gb - 1) / gb : 1;
  const long long total = N << ls;
  const unsigned nb = (unsigned)std::min<long long>((total + 255) / 256, 4096);
  for (int q = 0; q < ng; ++q) {
    const int c0 = q * gb, nc = j - c0 < gb ? j - c0 : gb;
    const int first = q == 0, last = q == ng - 1;
    const size_t lds = (size_t)2 * (nc > 0 ? nc : 0) * S * sizeof(cpx<double>);
    kb_dcgs_b<<<nb, 256, lds, st>>>(V, ldv, c0, nc, j, first, last, N, ls, K, lo);
    VHB_CHECK();
  }
  return hipSuccess;
}

hipError_t batch_finalize(BatchKrylovDev* K, int j, int S, hipStream_t st) {
  kb_finalize<<<1, 64, 0, st>>>(K, j, S);
  VHB_CHECK();
  return hipSuccess;
}
hipError_t batch_cycle_init(BatchKrylovDev* K, int m, int S, hipStream_t st) {
  kb_cycle_init<<<1, 64, 0, st>>>(K, m, S);
  VHB_CHECK();
  return hipSuccess;
}
hipError_t batch_backsolve(BatchKrylovDev* K, int S, hipStream_t st) {
  kb_backsolve<<<1, 64, 0, st>>>(K, S);
  VHB_CHECK();
  return hipSuccess;
}
hipError_t batch_update_x(const BatchKrylovDev* K, int kmax, int pz, const void* Z, size_t ldz,
                          cpx<double>* x, long long N, int ls, hipStream_t st) {
  const unsigned nb = nblk(N << ls, 256);
  if (pz == PREC_F64)
    kb_update_x<double><<<nb, 256, 0, st>>>(K, kmax, (const cpx<double>*)Z, ldz, x, N, ls);
  else
    kb_update_x<float><<<nb, 256, 0, st>>>(K, kmax, (const cpx<float>*)Z, ldz, x, N, ls);
  VHB_CHECK();
  return hipSuccess;
}
hipError_t batch_scale(const BatchKrylovDev* K, const cpx<double>* w, cpx<double>* v, long long N,
                       int ls, hipStream_t st) {
  kb_scale<<<nblk(N << ls, 256), 256, 0, st>>>(K, w, v, N, ls);
  VHB_CHECK();
  return hipSuccess;
}

}  // namespace vh
