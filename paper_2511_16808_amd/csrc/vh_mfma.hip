// vh_mfma.hip -- batched additive-Vanka sweep on the matrix cores (2D, Full 3x3 patch).
//
// With S sources sharing one hierarchy, the smoother of Sec. 3.2 (eq. (smoother)) is
// per patch c a dense complex product E_c = A_c^{-1} [r_c^(1) ... r_c^(S)] (9 x 9 times
// 9 x S), followed by the weighted overlap-add of E_c into the 9 member nodes.  Here the
// product runs on MFMA in its real embedding
//
//     [E_re; E_im] (18 x S) = [[Ar, -Ai], [Ai, Ar]] (18 x 18) . [R_re; R_im] (18 x S),
//
// (rows and columns interleaved (re, im) per patch member, the weights w_l / cnt already
// folded into the stored inverse rows), so that each lane ends with whole complex
// outputs of one source and the overlap-add is contiguous in the sources.  Two
// contractions are provided: FP32 (v_mfma_f32_16x16x4_f32, K = 18 in 5 steps of 4)
// and split BF16 (v_mfma_f32_16x16x32_bf16 on hi/lo halves, hi*hi + hi*lo + lo*hi,
// FP32 accumulation; the dropped lo*lo term is below 2^-16 relative).
//
// Data flow.  A block owns a strip of TX = TXP - 2 output columns and a chunk of rows,
// and marches down the rows: per patch row py it computes the TXP patches centred on
// columns x0-1 .. x0+TX (every patch that touches the strip), their member residuals
// read from a 3-row ring of the residual in LDS, their inverse rows staged in LDS by
// coalesced row loads, and adds E into a 3-row ring of FP32 accumulators in LDS.  Output
// row py-1 is complete after patch row py and is written out once.  Patches that are
// added at the same time are SUB = TXP/4 >= 4 columns apart (one per wavefront), so
// their member sets are disjoint: no atomics, and the order of the nine contributions
// to every node is fixed.  The next residual row and the next patch row's inverse rows
// are loaded into registers while the current row computes.
#include "vh_launch.h"

namespace vh {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int MW = 4;    // wavefronts per block
constexpr int NPM = 9;   // members of a Full 3x3 patch
constexpr int MPAD = 12; // member slots per staged inverse row (16-byte aligned runs of 4)

// (re, im) -> bf16 pair, re in the low half (round to nearest even)
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  const bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
// hi = bf16(x), lo = bf16(x - hi), for both halves of a complex number
__device__ __forceinline__ uint2 split_pair(float a, float b) {
  const unsigned h = bf16_pair(a, b);
  const float ah = __uint_as_float(h << 16), bh = __uint_as_float(h & 0xffff0000u);
  return make_uint2(h, bf16_pair(a - ah, b - bh));
}
__device__ __forceinline__ uint2 float_pair(float a, float b) {
  return make_uint2(__float_as_uint(a), __float_as_uint(b));
}

__device__ __forceinline__ bool inside2(const Grid& g, int x, int y) {
  return (unsigned)x < (unsigned)g.nx && (unsigned)y < (unsigned)g.ny;
}

}  // namespace

template <bool ZERO, int LS, bool SPLIT, int TXP>
__global__ __launch_bounds__(256) void kb_sweep_mfma(Grid g, int rows,
                                                     const cpx<float>* __restrict__ G,
                                                     const cpx<float>* __restrict__ r,
                                                     cpx<float>* __restrict__ u) {
  constexpr int S = 1 << LS, MT = S / 16;  // M tiles of 16 sources
  constexpr int TX = TXP - 2, RC = TXP + 2, SUB = TXP / MW;
  static_assert(SUB >= 3, "patches added together must be >= 3 columns apart");
  constexpr int NR = (RC * S + 255) / 256;           // residual row elements per thread
  constexpr int NG = (TXP * NPM * NPM + 255) / 256;  // inverse entries per thread
  __shared__ uint2 rr[3][RC][S];              // residual ring (split or FP32 bits)
  __shared__ __align__(16) uint2 gb[TXP][2][NPM][MPAD];  // B entries: patch, version ro, row a
  __shared__ float2 ua[3][TX][S];             // overlap-add accumulator ring
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nstrip = (g.nx + TX - 1) / TX;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % (unsigned)nstrip) * TX;
  const int yb = (int)(b / (unsigned)nstrip) * rows;
  if (yb >= g.ny) return;  // whole block
  const int ye = yb + rows < g.ny ? yb + rows : g.ny;
  const int py_lo = yb > 0 ? yb - 1 : 0, py_hi = ye < g.ny - 1 ? ye : g.ny - 1;
  const size_t Np = (size_t)g.Np;

  for (int e = tid; e < 3 * TX * S; e += 256) (&ua[0][0][0])[e] = make_float2(0.f, 0.f);
  for (int e = tid; e < TXP * 2 * NPM * MPAD; e += 256) (&gb[0][0][0][0])[e] = make_uint2(0, 0);

  cpx<float> rv[NR], gv[NG];
  auto load_row = [&](int y) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int e = tid + 256 * i, col = e >> LS, s = e & (S - 1);
      const int x = x0 - 2 + col;
      rv[i] = (e < RC * S && inside2(g, x, y)) ? r[((size_t)y * g.nx + x) * S + s]
                                                : cmk(0.f, 0.f);
    }
  };
  auto store_row = [&](int y) {
    uint2* dst = &rr[(y + 3) % 3][0][0];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int e = tid + 256 * i;
      if (e < RC * S)
        dst[e] = SPLIT ? split_pair(rv[i].re, rv[i].im) : float_pair(rv[i].re, rv[i].im);
    }
  };
  auto load_g = [&](int py) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int e = tid + 256 * i, p = e % TXP, q = e / TXP;
      const int a = q / NPM;
      const int px = x0 - 1 + p, x = px + a % 3 - 1, y = py + a / 3 - 1;
      gv[i] = (e < TXP * NPM * NPM && (unsigned)px < (unsigned)g.nx && inside2(g, x, y))
                  ? G[(size_t)q * Np + (size_t)x + (size_t)g.nxp * y]
                  : cmk(0.f, 0.f);
    }
  };
  auto store_g = [&]() {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int e = tid + 256 * i, p = e % TXP, q = e / TXP;
      if (e < TXP * NPM * NPM) {
        const int a = q / NPM, m = q % NPM;
        const float ar = gv[i].re, ai = gv[i].im;
        gb[p][0][a][m] = SPLIT ? split_pair(ar, -ai) : float_pair(ar, -ai);
        gb[p][1][a][m] = SPLIT ? split_pair(ai, ar) : float_pair(ai, ar);
      }
    }
  };

  load_row(py_lo - 1);
  store_row(py_lo - 1);
  load_row(py_lo);
  store_row(py_lo);
  load_row(py_lo + 1);
  load_g(py_lo);

  const int grp = lane >> 4, l16 = lane & 15;
  for (int py = py_lo; py <= py_hi; ++py) {
    __syncthreads();  // the previous row is done with ring slot (py + 1) % 3 and gb
    store_row(py + 1);
    store_g();
    __syncthreads();
    if (py < py_hi) {
      load_row(py + 2);
      load_g(py + 1);
    }
    for (int j = 0; j < SUB; ++j) {
      const int p = j + SUB * wv, px = x0 - 1 + p;
      if ((unsigned)px < (unsigned)g.nx) {  // uniform over the wavefront
        // MFMA operands: A = patch matrix, rows (a, ro) = 16 tm + l16 (tm = 1 holds only
        // a = 8), columns k = (m, ri); B = residuals, rows k, columns = sources 16 tn + l16.
        // Lane group grp holds k = 8 grp .. 8 grp + 7, i.e. members 4 grp .. 4 grp + 3.
        f32x4 acc[2][MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[0][t] = acc[1][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (SPLIT) {
          bf16x8 ah[2], al[2];
#pragma unroll
          for (int tm = 0; tm < 2; ++tm) {
            const int row = 16 * tm + l16, a = row >> 1, ro = row & 1;
            u32x4 h = {0, 0, 0, 0}, lo = {0, 0, 0, 0};
            if (a < NPM && grp < 3) {
              const uint4* src = reinterpret_cast<const uint4*>(&gb[p][ro][a][4 * grp]);
              const uint4 v0 = src[0], v1 = src[1];
              h = u32x4{v0.x, v0.z, v1.x, v1.z};
              lo = u32x4{v0.y, v0.w, v1.y, v1.w};
            }
            ah[tm] = __builtin_bit_cast(bf16x8, h);
            al[tm] = __builtin_bit_cast(bf16x8, lo);
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            const int s = 16 * t + l16;
            u32x4 h = {0, 0, 0, 0}, lo = {0, 0, 0, 0};
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int m = 4 * grp + jj;
              if (m < NPM) {
                const int dx = m % 3 - 1, dy = m / 3 - 1;
                const uint2 v = rr[(py + dy + 3) % 3][p + 1 + dx][s];
                h[jj] = v.x;
                lo[jj] = v.y;
              }
            }
            const bf16x8 bh = __builtin_bit_cast(bf16x8, h), bl = __builtin_bit_cast(bf16x8, lo);
#pragma unroll
            for (int tm = 0; tm < 2; ++tm) {
              acc[tm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[tm], bh, acc[tm][t], 0, 0, 0);
              acc[tm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm], bl, acc[tm][t], 0, 0, 0);
              acc[tm][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[tm], bh, acc[tm][t], 0, 0, 0);
            }
          }
        } else {
          // FP32: K = 18 in 5 steps of 4; lane holds k = 4 st + grp
#pragma unroll
          for (int st = 0; st < 5; ++st) {
            const int k = 4 * st + grp, m = k >> 1, ri = k & 1;
            float ak[2];
#pragma unroll
            for (int tm = 0; tm < 2; ++tm) {
              const int row = 16 * tm + l16, a = row >> 1, ro = row & 1;
              ak[tm] = 0.f;
              if (a < NPM && m < NPM) {
                const uint2 v = gb[p][ro][a][m];
                ak[tm] = __uint_as_float(ri ? v.y : v.x);
              }
            }
            const int dx = m % 3 - 1, dy = m / 3 - 1;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
              float bk = 0.f;
              if (m < NPM) {
                const uint2 v = rr[(py + dy + 3) % 3][p + 1 + dx][16 * t + l16];
                bk = __uint_as_float(ri ? v.y : v.x);
              }
#pragma unroll
              for (int tm = 0; tm < 2; ++tm)
                acc[tm][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ak[tm], bk, acc[tm][t], 0, 0, 0);
            }
          }
        }
        // overlap-add: lane holds rows 16 tm + 4 grp + i of E, i.e. (re, im) of outputs
        // a = 8 tm + 2 grp and a + 1, for source 16 t + l16: contiguous float2 runs
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
#pragma unroll
          for (int h2 = 0; h2 < 2; ++h2) {
            const int a = 8 * tm + 2 * grp + h2;
            if (a < NPM) {
              const int x = px + a % 3 - 1, y = py + a / 3 - 1;
              if (x >= x0 && x < x0 + TX && x < g.nx && y >= yb && y < ye) {
                float2* dst = &ua[y % 3][x - x0][0];
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                  float2& d = dst[16 * t + l16];
                  d = make_float2(d.x + acc[tm][t][2 * h2], d.y + acc[tm][t][2 * h2 + 1]);
                }
              }
            }
          }
        }
      }
      __syncthreads();
    }
    // output row py - 1 has all its contributions
    const int yo = py - 1;
    if (yo >= yb && yo < ye) {
      for (int e = tid; e < TX * S; e += 256) {
        const int col = e >> LS, s = e & (S - 1), x = x0 + col;
        float2& a = ua[yo % 3][col][s];
        if (x < g.nx) {
          cpx<float>& o = u[((size_t)yo * g.nx + x) * S + s];
          o = ZERO ? cmk(a.x, a.y) : cmk(o.re + a.x, o.im + a.y);
        }
        a = make_float2(0.f, 0.f);
      }
    }
  }
  // the last grid row has no patch row below it
  if (ye == g.ny && py_hi == g.ny - 1) {
    const int yo = g.ny - 1;
    if (yo >= yb) {
      for (int e = tid; e < TX * S; e += 256) {
        const int col = e >> LS, s = e & (S - 1), x = x0 + col;
        if (x < g.nx) {
          const float2 a = ua[yo % 3][col][s];
          cpx<float>& o = u[((size_t)yo * g.nx + x) * S + s];
          o = ZERO ? cmk(a.x, a.y) : cmk(o.re + a.x, o.im + a.y);
        }
      }
    }
  }
}

namespace {

template <bool SPLIT, int TXP, int LS>
hipError_t launch_mfma(Grid g, int rows, const void* G, const void* r, void* u, bool zero,
                       hipStream_t st) {
  constexpr int TX = TXP - 2;
  const long long nstrip = (g.nx + TX - 1) / TX, nchunk = (g.ny + rows - 1) / rows;
  const unsigned nb = (unsigned)(nstrip * nchunk);
  auto Gp = (const cpx<float>*)G;
  auto rp = (const cpx<float>*)r;
  auto up = (cpx<float>*)u;
  if (zero)
    kb_sweep_mfma<true, LS, SPLIT, TXP><<<nb, 256, 0, st>>>(g, rows, Gp, rp, up);
  else
    kb_sweep_mfma<false, LS, SPLIT, TXP><<<nb, 256, 0, st>>>(g, rows, Gp, rp, up);
  return hipGetLastError();
}

template <bool SPLIT, int TXP>
hipError_t launch_mfma_ls(Grid g, int ls, int rows, const void* G, const void* r, void* u,
                          bool zero, hipStream_t st) {
  if (ls == 4) return launch_mfma<SPLIT, TXP, 4>(g, rows, G, r, u, zero, st);
  if (ls == 5) return launch_mfma<SPLIT, TXP, 5>(g, rows, G, r, u, zero, st);
  return launch_mfma<SPLIT, TXP, 6>(g, rows, G, r, u, zero, st);
}

}  // namespace

hipError_t batch_sweep_mfma(Grid g, int ls, int split, int txp, int rows, const void* G,
                            const void* r, void* u, bool zero, hipStream_t st) {
  if (g.dim != 2 || ls < 4 || ls > 6 || rows < 1 || (txp != 16 && txp != 32))
    return hipErrorInvalidValue;
  if (split) {
    if (txp == 16) return launch_mfma_ls<true, 16>(g, ls, rows, G, r, u, zero, st);
    return launch_mfma_ls<true, 32>(g, ls, rows, G, r, u, zero, st);
  }
  if (txp == 16) return launch_mfma_ls<false, 16>(g, ls, rows, G, r, u, zero, st);
  return launch_mfma_ls<false, 32>(g, ls, rows, G, r, u, zero, st);
}

}  // namespace vh
