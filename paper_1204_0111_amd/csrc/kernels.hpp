// Host-side launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_ext.h>

#include "devtypes.hpp"
#include "plan.hpp"

namespace hsw {

// Events that the launches record (hipExtLaunchKernelGGL), set by the driver
// while a kernel class is timed: `start` at the start of the first launch
// after it is set (the launch clears it), `stop` at the end of every launch,
// so a group of launches (a pass and its finishing launch) is timed whole.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming& launch_timing();

}  // namespace hsw

#define HSW_LAUNCH(KERNEL, GRID, BLOCK, SHM, STREAM, ...)                                     \
    do {                                                                                     \
        ::hsw::LaunchTiming& lt_ = ::hsw::launch_timing();                                   \
        if (lt_.stop) {                                                                      \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, lt_.start, lt_.stop, 0,  \
                                  __VA_ARGS__);                                              \
            lt_.start = nullptr;                                                             \
        } else {                                                                             \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);               \
        }                                                                                    \
    } while (0)

namespace hsw {

// factor.hip
template <typename T>
void launch_assemble(const int2* work, int nwork, const FrontInst* inst, const PanelDev* pan,
                     const ProbDev* prob, const int* perm, const int* ulist, const int* cmap,
                     const Cx<double>* et, Cx<T>* Lb, Cx<T>* Wcur, const Cx<T>* Wchild,
                     hipStream_t st);
template <typename T>
void launch_ldlt_diag(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* dinv,
                      int k, int* err, hipStream_t st);
template <typename T>
void launch_panel_trsm(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb,
                       const Cx<T>* dinv, int k, hipStream_t st);
// mode: 0 right-looking trailing update of pivot block k, 1 left-looking
// update of block column k, 2 final Schur update of F_BR (see factor.hip)
template <typename T>
void launch_update(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* Wcur, int k,
                   int mode, int bf16, hipStream_t st);
template <typename T>
void launch_inverse(const int2* work, int nwork, const FrontInst* inst, const Cx<T>* Lb, Cx<T>* Gb,
                    Cx<T>* Tb, hipStream_t st);
template <typename T>
void launch_lf_copy(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, const Cx<T>* Tb,
                    hipStream_t st);

// solve.hip
template <typename T>
void launch_fwd(const PassArgs<T>& A, int nwork, int rb, int smax, int nmax, hipStream_t st);
template <typename T>
void launch_bwd(const PassArgs<T>& A, int nwork, int cb, int nmax, hipStream_t st);
// forward matrix-core pass: form 0 / 3 (items of 64 rows, 4 / 8 waves splitting
// the contraction), 1 / 4 (items of 16 rows, 4 / 8 waves), 2 (row-split, items
// of 64 rows, fwd_rs_lds_bytes(smax) bytes of LDS per workgroup), 5 (items of
// 64 rows, contraction split over A.nsplit workgroups; A.part holds
// nwork x groups x nsplit x 1024 partial entries), 6 (as 5 for items of 16
// rows, 256 partial entries each) or 7 (items of 16 rows, 2 waves)
template <typename T>
void launch_fwd_mm(const PassArgs<T>& A, int nwork, int form, int smax, hipStream_t st);
template <typename T>
size_t fwd_rs_lds_bytes(int smax);
// the panel's right-hand side into h2, in elimination order (matrix-core passes)
template <typename T>
void launch_rhs_scatter(const PassArgs<T>& A, hipStream_t st);
// backward matrix-core pass: form 0 (items of 64 columns, 4 waves), 1 / 2 / 3
// (items of 16 columns, 4 / 8 / 16 waves; complex128: 8), 4 (items of 64
// columns, contraction split over A.nsplit workgroups, as forward form 5) or
// 5 / 6 (as 1 / 2, four chunks in flight per wave), 7 (as 4 for items of 16
// columns) or 8 (items of 16 columns, 2 waves)
template <typename T>
void launch_bwd_mm(const PassArgs<T>& A, int nwork, int form, hipStream_t st);
template <typename T>
int solve_rhs_chunk(int nrhs, int nmax);
// triangular passes with the kept factors (fwd: forward pass, else backward),
// one work item per front
template <typename T>
void launch_tri(const PassArgs<T>& A, int nwork, int nmax, bool fwd, hipStream_t st);

// assemble.hip
void launch_axis_table(Cx<double>* out, int nj, int gj, double h, double C, double omega,
                       hipStream_t st);
void launch_aux_table(Cx<double>* out, int n3, int g, int lo, int ga, int nz, double h, double C,
                      double omega, hipStream_t st);
void launch_check_velocity(const double* c, int64_t n, int* bad, hipStream_t st);

// krylov.hip
// active (per right-hand side) and run: see k_matvec; NULL for all
void launch_matvec(const ProbDev& Q, const Cx<double>* et, const Cx<double>* x, Cx<double>* y,
                   const Cx<double>* b, int64_t ld, int nrhs, int mode, hipStream_t st,
                   const int* active = nullptr, const int* run = nullptr);
int dots_chunks(int64_t N);
void launch_dots(const Cx<double>* V, int64_t vstride, const Cx<double>* w, int64_t ld, int64_t N,
                 int nvec, int nrhs, const int* active, Cx<double>* partial, Cx<double>* h, int hld,
                 Cx<double>* hout, int mode, hipStream_t st);
void launch_axpy_multi(const Cx<double>* V, int64_t vstride, Cx<double>* w, int64_t ld, int64_t N,
                       int nvec, const Cx<double>* coef, int cld, const int* nvec_rhs,
                       const int* active, int mode, int nrhs, hipStream_t st);
// w -= V coef (coef as written by launch_dots), then h += V^H w with the new
// w (and hout := those products): launch_axpy_multi and launch_dots (mode 1)
// in one pass over the basis
void launch_axpy_dots(const Cx<double>* V, int64_t vstride, Cx<double>* w, int64_t ld, int64_t N, int nvec,
                      const Cx<double>* coef, int cld, int nrhs, const int* active, Cx<double>* partial,
                      Cx<double>* h, int hld, Cx<double>* hout, hipStream_t st);
void launch_norm(const Cx<double>* w, int64_t ld, int64_t N, int nrhs, const int* active,
                 double* partial, double* norm, Cx<double>* hptr, int hld, hipStream_t st);
void launch_scale(const Cx<double>* w, Cx<double>* v, int64_t ld, int64_t N, int nrhs,
                  const double* norm, const int* active, hipStream_t st);
void launch_givens(int j, int k, int nrhs, Cx<double>* H, double* cs, Cx<double>* sn,
                   Cx<double>* g, const double* bnorm, double* est, const int* active,
                   hipStream_t st);
void launch_lsq(int k, int nrhs, const Cx<double>* H, const Cx<double>* g, const int* jcount,
                Cx<double>* y, hipStream_t st);
// z := x (nrhs columns of N entries, stride ld), skipped while *run is 0
void launch_copy_cols(const Cx<double>* x, Cx<double>* z, int64_t ld, int64_t N, int nrhs, const int* run,
                      hipStream_t st);
// GMRES convergence test on the device after Arnoldi step j (k_conv)
void launch_conv(int j, int nrhs, const double* est, double rtol, int maxit, int* active, int* iters,
                 int* jcount, int* run, hipStream_t st);
void launch_cycle_init(int k, int nrhs, const double* beta, Cx<double>* g, const int* active,
                       hipStream_t st);

// bkrylov.hip (block GMRES; blocks of at most 16 vectors)
constexpr int BLOCK_KRYLOV_MAX = 16;
int bdots_chunks(int64_t N);
void launch_bdots(const Cx<double>* Q, int64_t qld, int m, const Cx<double>* W, int64_t wld, int q,
                  int64_t N, Cx<double>* partial, Cx<double>* out, hipStream_t st);
void launch_bcombine(const Cx<double>* Q, int64_t qld, int m, const Cx<double>* C, int q,
                     Cx<double>* X, int64_t ld, const int* col, int64_t N, double alpha, double beta,
                     hipStream_t st);

}  // namespace hsw
