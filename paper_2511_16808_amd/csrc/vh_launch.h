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

hipError_t fill(void* p, size_t n, int prec, double re, double im, hipStream_t s);
hipError_t convert(const void* a, int pa, void* b, int pb, size_t n, hipStream_t s);
hipError_t fine_operator(int dim, Grid g, const double* kappa, const double* gamma, double h,
                         double omega, double alpha, int bc, int sw, double samp, cpx<double>* H,
                         cpx<double>* Hs, hipStream_t s);
hipError_t check_media(long long N, const double* kappa, const double* gamma, int* flag,
                       hipStream_t s);
hipError_t stencil(int dim, int shape, Grid g, int mode, int pc, const void* A, int px,
                   const void* x, int py, const void* b, void* y, hipStream_t s);
// form: 0 = per-patch Full (Np*Np entries), 1 = per-patch point, 2 = assembled 5^dim box
hipError_t vanka_sweep(int dim, int form, Grid g, int prec, const void* G, const void* r, void* u,
                       bool zero, hipStream_t s);
hipError_t vanka_setup(int dim, int shape, int patch, Grid g, const cpx<double>* A, double w,
                       int prec, void* G, hipStream_t s);
hipError_t vanka_assemble(int dim, Grid g, int prec, const void* G, void* B, hipStream_t s);
hipError_t galerkin(int dim, int sin, int sout, int rf, int pf, Grid gf, Grid gc,
                    const cpx<double>* Af, cpx<double>* Ac, hipStream_t s);
hipError_t restrict_(int dim, int rf, Grid gf, Grid gc, int prec, const void* r, void* rc,
                     hipStream_t s);
hipError_t prolong_add(int dim, int pf, Grid gf, Grid gc, int prec, const void* e, void* u,
                       hipStream_t s);
hipError_t dense_assemble(int dim, int shape, Grid g, const cpx<double>* A, cpx<double>* D,
                          hipStream_t s);
hipError_t gj_invert(int n, cpx<double>* M, int* perm, cpx<double>* col, hipStream_t s);
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

}  // namespace vh
