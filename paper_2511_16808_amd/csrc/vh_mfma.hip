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

// Workgroup barrier that orders LDS only: global loads issued before it (the next
// row's prefetch) stay in flight across it, where __syncthreads would wait for them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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
  constexpr int S = 1 << LS, MT = S / 16;  // source tiles of 16
  constexpr int TX = TXP - 2, RC = TXP + 2, SUB = TXP / MW;
  static_assert(SUB >= 3, "patches added together must be >= 3 columns apart");
  constexpr int SP = S + 2;            // LDS stride of one node (16 B of padding)
  constexpr int RS = RC * SP;          // residual ring: stride of one row
  constexpr int US = TX * SP;          // accumulator ring: stride of one row
  constexpr int NROW = 2 * NPM;        // rows (a, ro) of the embedded inverse
  constexpr int GPS = 3 * NROW * 4 + 2;  // staged inverse of one patch: [grp][row][4]
  constexpr int NR = (RC * S + 255) / 256;           // residual row elements per thread
  constexpr int NG = (TXP * NPM * NPM + 255) / 256;  // inverse entries per thread
  constexpr int ZR = 3 * RS;           // S zero residuals (members outside the patch)
  constexpr int ZA = TXP * GPS;        // 4 zero inverse entries (rows past the 18)
  constexpr int NU = (TX * S + 255) / 256;  // output row elements per thread
  __shared__ uint2 rr[3 * RS + S];                 // residual ring (split or FP32 bits)
  __shared__ __align__(16) uint2 gb[TXP * GPS + 4];  // A operands per patch
  __shared__ float2 ua[3 * US];                    // overlap-add ring
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int grp = lane >> 4, l16 = lane & 15;
  const int nstrip = (g.nx + TX - 1) / TX;
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % (unsigned)nstrip) * TX;
  const int yb = (int)(b / (unsigned)nstrip) * rows;
  if (yb >= g.ny) return;  // whole block
  const int ye = yb + rows < g.ny ? yb + rows : g.ny;
  const int xe = x0 + TX < g.nx ? x0 + TX : g.nx;
  const int py_lo = yb > 0 ? yb - 1 : 0, py_hi = ye < g.ny - 1 ? ye : g.ny - 1;
  const size_t rowS = (size_t)g.nx * S;  // elements of one grid row of a batch vector

  for (int e = tid; e < 3 * US; e += 256) ua[e] = make_float2(0.f, 0.f);
  for (int e = tid; e < TXP * GPS + 4; e += 256) gb[e] = make_uint2(0, 0);
  for (int e = tid; e < S; e += 256) rr[ZR + e] = make_uint2(0, 0);

  // ---- per-lane operand constants
  // A operand (inverse rows): row 16 tm + l16 of the 18 rows; the split form reads members
  // 4 grp .. 4 grp + 3 (grp 3 only padding), the FP32 form one (m, ri) per step.  Lanes
  // without a row read the zero block.
  int arow[2];
  bool aok[2];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
    const int row = 16 * tm + l16;
    aok[tm] = row < NROW && (!SPLIT || grp < 3);
    arow[tm] = ((SPLIT ? grp : 0) * NROW + row) * 4;
  }
  // B operand (member residuals): member m = 4 grp + jj (split) or (4 st + grp) / 2;
  // members past the ninth read the zero residuals
  constexpr int NB = SPLIT ? 4 : 5;
  int bdx[NB], bdy[NB];
  bool bok[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int m = SPLIT ? 4 * grp + k : (4 * k + grp) >> 1;
    const int mc = m < NPM ? m : NPM - 1;
    bdx[k] = mc % 3 - 1;
    bdy[k] = mc / 3 - 1;
    bok[k] = m < NPM;
  }
  // outputs a = 8 tm + 2 grp + h2 held by this lane
  int odx[2][2], ody[2][2];
  bool ook[2][2];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int a = 8 * tm + 2 * grp + h2, ac = a < NPM ? a : NPM - 1;
      odx[tm][h2] = ac % 3 - 1;
      ody[tm][h2] = ac / 3 - 1;
      ook[tm][h2] = a < NPM;
    }

  // ---- per-thread staging constants (the rows change, the columns do not)
  int r_goff[NR], r_ldst[NR];
  bool r_ok[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int e = tid + 256 * i, col = e >> LS, sl = e & (S - 1), x = x0 - 2 + col;
    r_ok[i] = e < RC * S && (unsigned)x < (unsigned)g.nx;
    r_goff[i] = x * S + sl;
    r_ldst[i] = col * SP + sl;
  }
  size_t g_goff[NG];
  int g_dy[NG], g_ldst[NG];
  bool g_ok[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int e = tid + 256 * i, p = e % TXP, q = e / TXP, a = q / NPM, m = q % NPM;
    const int px = x0 - 1 + p, x = px + a % 3 - 1;
    g_ok[i] = e < TXP * NPM * NPM && (unsigned)px < (unsigned)g.nx && (unsigned)x < (unsigned)g.nx;
    g_goff[i] = (size_t)q * g.Np + (size_t)(g_ok[i] ? x : 0);
    g_dy[i] = a / 3 - 1;
    g_ldst[i] = p * GPS + ((m >> 2) * NROW + 2 * a) * 4 + (m & 3);
  }
  int u_goff[NU], u_lsrc[NU];
  bool u_ok[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const int e = tid + 256 * i, col = e >> LS, sl = e & (S - 1), x = x0 + col;
    u_ok[i] = e < TX * S && x < g.nx;
    u_goff[i] = x * S + sl;
    u_lsrc[i] = col * SP + sl;
  }

  cpx<float> rv[NR], gv[NG], uv[NU];
  auto load_row = [&](int y) {
    const bool yok = (unsigned)y < (unsigned)g.ny;
#pragma unroll
    for (int i = 0; i < NR; ++i)
      rv[i] = (yok && r_ok[i]) ? r[(size_t)y * rowS + r_goff[i]] : cmk(0.f, 0.f);
  };
  auto store_row = [&](int y) {
    uint2* dst = rr + ((y + 3) % 3) * RS;
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (tid + 256 * i < RC * S)
        dst[r_ldst[i]] = SPLIT ? split_pair(rv[i].re, rv[i].im) : float_pair(rv[i].re, rv[i].im);
  };
  auto load_g = [&](int py) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int y = py + g_dy[i];
      gv[i] = (g_ok[i] && (unsigned)y < (unsigned)g.ny)
                  ? G[g_goff[i] + (size_t)g.nxp * (size_t)y]
                  : cmk(0.f, 0.f);
    }
  };
  // entry (a, m) -> rows (a, 0) = (Ar, -Ai) and (a, 1) = (Ai, Ar) at member slot m
  auto store_g = [&]() {
#pragma unroll
    for (int i = 0; i < NG; ++i)
      if (tid + 256 * i < TXP * NPM * NPM) {
        const float ar = gv[i].re, ai = gv[i].im;
        gb[g_ldst[i]] = SPLIT ? split_pair(ar, -ai) : float_pair(ar, -ai);
        gb[g_ldst[i] + 4] = SPLIT ? split_pair(ai, ar) : float_pair(ai, ar);
      }
  };
  const unsigned* rr32 = reinterpret_cast<const unsigned*>(rr);
  const unsigned* gb32 = reinterpret_cast<const unsigned*>(gb);

  load_row(py_lo - 1);
  store_row(py_lo - 1);
  load_row(py_lo);
  store_row(py_lo);
  load_row(py_lo + 1);
  load_g(py_lo);

  for (int py = py_lo; py <= py_hi; ++py) {
    lds_barrier();  // the previous row is done with ring slot (py + 1) % 3 and gb
    store_row(py + 1);
    store_g();
    lds_barrier();
    if (py < py_hi) {
      load_row(py + 2);
      load_g(py + 1);
    }
    const int yo = py - 1;  // output row completed by this patch row
    const bool fin = yo >= yb && yo < ye;
    if (!ZERO && fin) {
#pragma unroll
      for (int i = 0; i < NU; ++i)
        uv[i] = u_ok[i] ? u[(size_t)yo * rowS + u_goff[i]] : cmk(0.f, 0.f);
    }
    // ring offsets of this row: residual members, and kept outputs
    int rb[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      rb[k] = ((py + bdy[k] + 3) % 3) * RS + (1 + bdx[k]) * SP + l16;
    int ob[2][2];
    bool orow[2][2];
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int y = py + ody[tm][h2];
        orow[tm][h2] = ook[tm][h2] && y >= yb && y < ye;
        ob[tm][h2] = ((y + 3) % 3) * US + (odx[tm][h2] - x0) * SP + l16;
      }
    for (int j = 0; j < SUB; ++j) {
      const int p = j + SUB * wv, px = x0 - 1 + p;
      if ((unsigned)px < (unsigned)g.nx) {  // uniform over the wavefront
        f32x4 acc[2][MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[0][t] = acc[1][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        int ab[2], bb[NB];
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) ab[tm] = aok[tm] ? p * GPS + arow[tm] : ZA;
#pragma unroll
        for (int k = 0; k < NB; ++k) bb[k] = bok[k] ? rb[k] + p * SP : ZR + l16;
        if constexpr (SPLIT) {
          bf16x8 ah[2], al[2];
#pragma unroll
          for (int tm = 0; tm < 2; ++tm) {
            const uint4* src = reinterpret_cast<const uint4*>(gb + ab[tm]);
            const uint4 v0 = src[0], v1 = src[1];
            ah[tm] = __builtin_bit_cast(bf16x8, u32x4{v0.x, v0.z, v1.x, v1.z});
            al[tm] = __builtin_bit_cast(bf16x8, u32x4{v0.y, v0.w, v1.y, v1.w});
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            u32x4 h, lo;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const uint2 v = rr[bb[k] + 16 * t];
              h[k] = v.x;
              lo[k] = v.y;
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
          // K = 18 in 5 steps of 4: lane holds k = 4 st + grp, member k / 2, part k % 2
          // (k = 18, 19 fall on the zero padding of member slot 9)
          const int ri = grp & 1;
#pragma unroll
          for (int st = 0; st < 5; ++st) {
            const int m = (4 * st + grp) >> 1;
            float ak[2];
#pragma unroll
            for (int tm = 0; tm < 2; ++tm) {
              const int w = aok[tm] ? 2 * (ab[tm] + (m >> 2) * NROW * 4 + (m & 3)) + ri : 2 * ZA;
              ak[tm] = __uint_as_float(gb32[w]);
            }
#pragma unroll
            for (int t = 0; t < MT; ++t) {
              const float bk = __uint_as_float(rr32[2 * (bb[st] + 16 * t) + ri]);
#pragma unroll
              for (int tm = 0; tm < 2; ++tm)
                acc[tm][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ak[tm], bk, acc[tm][t], 0, 0, 0);
            }
          }
        }
        // overlap-add: lane holds (re, im) of outputs a = 8 tm + 2 grp + h2 for sources
        // 16 t + l16 (contiguous float2 runs); only lanes whose output node is kept touch
        // LDS (a = 9 .. 15 never exist, a = 8 lives in lane group 0)
#pragma unroll
        for (int tm = 0; tm < 2; ++tm)
#pragma unroll
          for (int h2 = 0; h2 < (tm == 0 ? 2 : 1); ++h2) {
            const int x = px + odx[tm][h2];
            if (orow[tm][h2] && x >= x0 && x < xe) {
              float2* dst = ua + ob[tm][h2] + px * SP;
#pragma unroll
              for (int t = 0; t < MT; ++t) {
                float2& d = dst[16 * t];
                d = make_float2(d.x + acc[tm][t][2 * h2], d.y + acc[tm][t][2 * h2 + 1]);
              }
            }
          }
      }
      lds_barrier();
    }
    // output row py - 1 has all its contributions
    if (fin) {
      float2* row = ua + (yo % 3) * US;
#pragma unroll
      for (int i = 0; i < NU; ++i) {
        if (tid + 256 * i < TX * S) {
          float2& a = row[u_lsrc[i]];
          if (u_ok[i])
            u[(size_t)yo * rowS + u_goff[i]] =
                ZERO ? cmk(a.x, a.y) : cmk(uv[i].re + a.x, uv[i].im + a.y);
          a = make_float2(0.f, 0.f);
        }
      }
    }
  }
  // the last grid row has no patch row below it
  if (ye == g.ny && py_hi == g.ny - 1) {
    const int yo = g.ny - 1;
    if (yo >= yb) {
      const float2* row = ua + (yo % 3) * US;
      for (int e = tid; e < TX * S; e += 256) {
        const int col = e >> LS, s = e & (S - 1), x = x0 + col;
        if (x < g.nx) {
          const float2 a = row[col * SP + s];
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
