// vh_launch.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include <algorithm>

#include "vh_common.h"

namespace vh {

enum Prec : int { PREC_F64 = 0, PREC_F32 = 1 };
enum OpMode : int { OP_APPLY = 0, OP_RESID = 1, OP_ADD = 2 };
enum Bc : int { BC_ABC = 0, BC_DIRICHLET = 1 };

constexpr int MMAX = 64;  // largest FGMRES restart length

// Device-resident state of one FGMRES cycle (FP64).
struct KrylovDev {
  cpx<double> H[MMAX * (MMAX + 1)];  // Hessenberg, column j at H + j*(MMAX+1)
  double cs[MMAX];
  cpx<double> sn[MMAX];
  cpx<double> g[MMAX + 1];
  cpx<double> y[MMAX];
  cpx<double> h1[MMAX + 1];
  cpx<double> h2[MMAX + 1];
  cpx<double> nrm2[1];
  double status[4];  // |g_{j+1}|, ||w||, breakdown flag, beta of the cycle
  double inv_nrm;
};

// Device-resident FGMRES state of a batch of up to 64 sources (FP64); every array
// is source-fastest with a stride of 64.
constexpr int DG = 12;  // basis columns per group of the delayed reduction pass
constexpr int PA_ROWS = 2 * DG + 3;            // pass-A sums per column group
constexpr int PA_GROUPS = (MMAX + DG) / DG;    // column groups of j <= MMAX

struct BatchKrylovDev {
  cpx<double> H[MMAX * (MMAX + 1) * 64];
  double cs[MMAX * 64];
  cpx<double> sn[MMAX * 64];
  cpx<double> g[(MMAX + 1) * 64];
  cpx<double> y[MMAX * 64];
  cpx<double> h1[(MMAX + 1) * 64];
  cpx<double> h2[(MMAX + 1) * 64];
  cpx<double> nrm2[64];
  double status[64 * 4];  // per source: |g_{j+1}|, ||w||, breakdown flag, beta
  double inv_nrm[64];
  int kcols[64];          // columns used by the next solution update (0 = frozen source)
  // delayed reorthogonalisation (one reduction pass and one update pass per step)
  cpx<double> pa[PA_GROUPS * PA_ROWS * 64];  // pass-A sums, column group q at rows q*PA_ROWS
  cpx<double> cprev[(MMAX + 1) * 64];  // first-pass coefficients of the last A z
  double nuprev[64];                   // norm of its lagged residual
  cpx<double> xb[MMAX * 64];           // pass B: v_j = (u - sum xb_i v_i) * ib
  cpx<double> yd[MMAX * 64];           //   u' = (w - sum yd_i v_i - gam u) * inu
  cpx<double> gam[64];
  double ib[64], inu[64];
};

hipError_t fill(void* p, size_t n, int prec, double re, double im, hipStream_t s);
hipError_t convert(const void* a, int pa, void* b, int pb, size_t n, hipStream_t s);
hipError_t fine_operator(int dim, Grid g, const double* kappa, const double* gamma, double h,
                         double omega, double alpha, int bc, int sw, double samp, cpx<double>* H,
                         cpx<double>* Hs, hipStream_t s);
// compact 4th-order fine operator (3^dim-box arrays), same arguments as fine_operator
hipError_t fine_compact4(int dim, Grid g, const double* kappa, const double* gamma, double h,
                         double omega, double alpha, int bc, int sw, double samp, cpx<double>* H,
                         cpx<double>* Hs, hipStream_t s);
hipError_t check_media(long long N, const double* kappa, const double* gamma, int* flag,
                       hipStream_t s);
hipError_t stencil(int dim, int shape, Grid g, int mode, int pc, const void* A, int px,
                   const void* x, int py, const void* b, void* y, hipStream_t s);
// form: 0 = per-patch Full (Np*Np entries), 1 = per-patch point, 2 = assembled 5^dim box
hipError_t vanka_sweep(int dim, int form, Grid g, int prec, const void* G, const void* r, void* u,
                       bool zero, hipStream_t s);
// u_out = u_in + B (q - A u_in) in one launch, where fused_sweep_ok(dim, form, shape); form
// 6 is the symmetric half (w its damping); u_out must not be u_in
bool fused_sweep_ok(int dim, int form, int shape);
hipError_t vanka_sweep_fused(int dim, int form, int shape, Grid g, int prec, const void* G,
                             double w, const void* A, const void* q, const void* u_in, void* u_out,
                             hipStream_t s);
// A slab of the smoother setup: patches centred at nodes [c_lo, c_hi) (unpadded linear
// index) write their rows to G[e * gstride + (padded member index - gbase)].  The whole
// grid is {0, N, 0, Np}.
struct Slab {
  long long c_lo, c_hi;
  long long gbase;
  size_t gstride;
};
// nopiv: eliminate in the natural order without pivoting (Full patch; for complex symmetric
// patch matrices with a positive definite imaginary part, where no pivot can vanish)
hipError_t vanka_setup(int dim, int shape, int patch, Grid g, const cpx<double>* A, double w,
                       int prec, void* G, Slab sl, hipStream_t s, bool nopiv = false);
hipError_t sample(Grid g, int E, int padded, int prec, int count, const long long* nodes,
                  const void* src, cpx<double>* out, hipStream_t s);
hipError_t unpad(Grid g, int E, int prec, const void* src, cpx<double>* dst, hipStream_t s);
// symmetric half of the assembled Full-patch smoother (upper half of the 5^d box, divided
// by the weights w / cnt_i): assembly, sweep, and the full stencil rebuilt for export
hipError_t vanka_assemble_sym(int dim, Grid g, int prec, const void* G, Slab sl, double w, void* S,
                              hipStream_t s);
// the sweep reads up to sym_guard(g) entries before plane 0: S must be preceded by that
// many zero entries of the same allocation, and followed by sym_tail(g) of them
long long sym_guard(const Grid& g);
long long sym_tail(const Grid& g);
// 3D: planes < 0 sweeps one plane per block, planes >= 2 walks that many planes per block
// (the mirrored entries of a plane come from the caches), 0 takes sym_walk_planes(g): the
// walk of SYM_WALK_PLANES planes when it still gives SYM_WALK_MIN_BLOCKS blocks.  The walk
// needs `carry`, device scratch of sym_carry_elems(g, planes) complex entries at the
// preconditioner precision (the mirrored sums handed from one chunk of planes to the next)
constexpr int SYM_WALK_PLANES = 6, SYM_WALK_MIN_BLOCKS = 1024;
int sym_walk_planes(const Grid& g);
long long sym_carry_elems(const Grid& g, int planes);
hipError_t vanka_sweep_sym(int dim, Grid g, int prec, const void* S, double w, const void* r,
                           void* u, bool zero, hipStream_t s, int planes = 0,
                           void* carry = nullptr);
hipError_t unpad_sym(Grid g, double w, int prec, const void* S, cpx<double>* dst, hipStream_t s);
hipError_t sample_sym(Grid g, double w, int prec, int count, const long long* nodes, const void* S,
                      cpx<double>* out, hipStream_t s);
// B rows of nodes [sl.c_lo, sl.c_hi) from the per-patch rows held as in vanka_setup
hipError_t vanka_assemble(int dim, int patch, Grid g, int prec, const void* G, Slab sl, void* B,
                          hipStream_t s);
hipError_t galerkin(int dim, int sin, int sout, int rf, int pf, Grid gf, Grid gc,
                    const cpx<double>* Af, cpx<double>* Ac, hipStream_t s);
hipError_t restrict_(int dim, int rf, Grid gf, Grid gc, int prec, const void* r, void* rc,
                     hipStream_t s);
// u = u_in + P e (u_in = nullptr: in place, u += P e)
hipError_t prolong_add(int dim, int pf, Grid gf, Grid gc, int prec, const void* e, void* u,
                       hipStream_t s, const void* u_in = nullptr);
// rc = R (q - A u) in one launch, where fused_restrict_ok(dim, rf, shape)
bool fused_restrict_ok(int dim, int rf, int shape);
hipError_t resid_restrict(int dim, int rf, int shape, Grid gf, Grid gc, int prec, const void* A,
                          const void* q, const void* u, void* rc, hipStream_t s);
hipError_t dense_assemble(int dim, int shape, Grid g, const cpx<double>* A, cpx<double>* D,
                          hipStream_t s);
// in-place inverse of the n x n row-major FP64 matrix M; work holds gj_workspace_bytes(n)
size_t gj_workspace_bytes(int n);
hipError_t gj_invert(int n, cpx<double>* M, void* work, hipStream_t s);
hipError_t dense_matvec(int n, const cpx<double>* D, int prec, const void* x, void* y,
                        hipStream_t s);
hipError_t cgs_pass(int mode, const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                    cpx<double>* w, size_t N, cpx<double>* part, int nb, cpx<double>* out,
                    hipStream_t s);
hipError_t arnoldi_finalize(KrylovDev* K, int j, int ldh, hipStream_t s);
hipError_t backsolve(KrylovDev* K, int k, int ldh, hipStream_t s);
hipError_t update_x(const KrylovDev* K, int k, int pz, const void* Z, size_t ldz, cpx<double>* x,
                    size_t N, hipStream_t s);
hipError_t scale_vec(const double* scale, const cpx<double>* w, cpx<double>* v, size_t N,
                     hipStream_t s);
hipError_t cycle_init(KrylovDev* K, int m, hipStream_t s);

// multi-source (batched) path, vectors [node][S], S = 1 << ls <= 64
hipError_t batch_gather(long long N, int S, int nsrc, const cpx<double>* q, cpx<double>* Q,
                        hipStream_t st);
hipError_t batch_scatter(long long N, int S, int nsrc, const cpx<double>* X, cpx<double>* u,
                         hipStream_t st);
// tile: the 64-source 2D sweep and stencil variant, 1 .. S64_TILES (0 = the default);
// ignored by every other form and batch width
constexpr int S64_TILES = 10;
constexpr int S64_DEFAULT_TILE = 7;
// tile: the 64-source 2D variant as for batch_sweep (0 = the default)
hipError_t batch_stencil(int dim, int shape, Grid g, int ls, int mode, int pc, const void* A,
                         int px, const void* x, int py, const void* b, void* y, hipStream_t st,
                         int tile = 0);
// batched 2D Full-patch sweep on MFMA (1 << ls sources, ls in 4..6, complex64):
// split = 0 FP32, 1 split BF16; txp = 16 or 32 patches per strip row; rows per block
hipError_t batch_sweep_mfma(Grid g, int ls, int split, int txp, int rows, const void* G,
                            const void* r, void* u, bool zero, hipStream_t st);
hipError_t batch_sweep(int dim, int form, Grid g, int ls, int prec, const void* G, const void* r,
                       void* u, bool zero, hipStream_t st, int tile = 0);
hipError_t batch_restrict(int dim, int rf, Grid gf, Grid gc, int ls, int prec, const void* r,
                          void* rc, hipStream_t st);
hipError_t batch_prolong_add(int dim, int pf, Grid gf, Grid gc, int ls, int prec, const void* e,
                             void* u, hipStream_t st);
hipError_t batch_dense(int n, int ls, const cpx<double>* D, int prec, const void* X, void* Y,
                       hipStream_t st);
hipError_t batch_cgs(int mode, const cpx<double>* V, size_t ldv, int nv, const cpx<double>* h,
                     cpx<double>* w, long long N, int ls, cpx<double>* part, int nb,
                     cpx<double>* out, hipStream_t st);
hipError_t batch_finalize(BatchKrylovDev* K, int j, int S, hipStream_t st);
hipError_t batch_cycle_init(BatchKrylovDev* K, int m, int S, hipStream_t st);
hipError_t batch_backsolve(BatchKrylovDev* K, int S, hipStream_t st);
hipError_t batch_update_x(const BatchKrylovDev* K, int kmax, int pz, const void* Z, size_t ldz,
                          cpx<double>* x, long long N, int ls, hipStream_t st);
hipError_t batch_scale(const BatchKrylovDev* K, const cpx<double>* w, cpx<double>* v, long long N,
                       int ls, hipStream_t st);
// delayed classical Gram-Schmidt with reorthogonalisation, step j: pass A reduces the
// dots of the final columns 0..j-1 with u = V_j (the lagged vector) and with
// w = V_wcol, and u^H w, u^H u, w^H w, into K->pa; dcgs_fin completes Hessenberg column
// j-1 (closing = 1: only that) and prepares pass B, which writes the final v_j into V_j
// and the next lagged vector into V_{j+1}
hipError_t batch_dcgs_a(const cpx<double>* V, size_t ldv, int j, int wcol, long long N, int ls,
                        cpx<double>* part, int nb, BatchKrylovDev* K, hipStream_t st);
hipError_t batch_dcgs_fin(BatchKrylovDev* K, int j, int S, int closing, hipStream_t st);
// lo (optional): also receives the new lagged vector rounded to complex64, the next
// preconditioner input
hipError_t batch_dcgs_b(cpx<double>* V, size_t ldv, int j, long long N, int ls,
                        const BatchKrylovDev* K, cpx<float>* lo, hipStream_t st);

}  // namespace vh
