// FP64 kernels of the GMRES(k) driver (Sec. 2.4): the 7-point mat-vec with
// the undamped operator A, and the Arnoldi / least-squares pieces.
//
// Reductions are two-stage with a fixed order (per-workgroup partial sums,
// then one pass over the partials), so results are bitwise reproducible.
// Vectors are complex128 on the padded grid; right-hand side r of a block
// starts at r * ld.  Per-right-hand-side state (Hessenberg matrix, rotations,
// residual estimate, activity flag) lives on the device.
#include "devtypes.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace hsw {

using C64 = Cx<double>;

// y = A x (mode 0) or y = b - A x (mode 1), coefficients from the stretch
// tables.  Right-hand sides with active[r] == 0 are skipped, and nothing is
// done while *run is 0 (active and run may be NULL).
__global__ __launch_bounds__(256) void k_matvec(ProbDev Q, const C64* __restrict__ et,
                                                const C64* __restrict__ x, C64* __restrict__ y,
                                                const C64* __restrict__ b, int64_t ld, int nrhs,
                                                int mode, const int* __restrict__ active,
                                                const int* __restrict__ run) {
    if (run && !*run) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= Q.Npad) return;
    const int N1 = Q.N[0], N2 = Q.N[1], N3 = Q.N[2];
    const int64_t N12 = (int64_t)N1 * N2;
    const int a3 = (int)(p / N12);
    const int rem = (int)(p - (int64_t)a3 * N12);
    const int a2 = rem / N1, a1 = rem - a2 * N1;
    const C64* e3n = et + Q.e_off[2];
    const C64* ie3 = et + Q.e_off[2] + N3;
    const NodeStretch st = node_stretch(Q, et, a1, a2, e3n, ie3, a3);
    const double inv_h2 = 1.0 / (Q.h * Q.h);
    const double c = velocity_at(Q, a1, a2, a3);
    const C64 dg = diag_entry(st, c, cx<double>(Q.omega * Q.omega, 0.0), inv_h2);
    C64 cm[3], cp[3];
    for (int j = 0; j < 3; ++j) {
        const C64 P = axis_weight(st, j);
        cm[j] = scale(P * st.im[j], -inv_h2);
        cp[j] = scale(P * st.ip[j], -inv_h2);
    }
    const bool h1m = a1 > 0, h1p = a1 + 1 < N1, h2m = a2 > 0, h2p = a2 + 1 < N2;
    const bool h3m = a3 > 0, h3p = a3 + 1 < N3;
    for (int r = 0; r < nrhs; ++r) {
        if (active && !active[r]) continue;
        const C64* xr = x + r * ld + p;
        C64 acc = dg * xr[0];
        if (h1m) cfma(acc, cm[0], xr[-1]);
        if (h1p) cfma(acc, cp[0], xr[1]);
        if (h2m) cfma(acc, cm[1], xr[-N1]);
        if (h2p) cfma(acc, cp[1], xr[N1]);
        if (h3m) cfma(acc, cm[2], xr[-N12]);
        if (h3p) cfma(acc, cp[2], xr[N12]);
        y[r * ld + p] = mode == 0 ? acc : b[r * ld + p] - acc;
    }
}

void launch_matvec(const ProbDev& Q, const C64* et, const C64* x, C64* y, const C64* b, int64_t ld,
                   int nrhs, int mode, hipStream_t st, const int* active, const int* run) {
    const int64_t nb = (Q.Npad + 255) / 256;
    HSW_LAUNCH(k_matvec, dim3((unsigned)nb), dim3(256), 0, st, Q, et, x, y, b, ld, nrhs, mode, active, run);
}

// ---------------------------------------------------------------------------
// Block sum of 256 complex values held one per thread; result valid in thread 0.
__device__ inline C64 block_sum(C64 v, C64* sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    C64 t = cx<double>(0, 0);
    if (tid == 0) t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return t;
}

// partial[(r * nchunk + chunk) * nvec + i] = sum over the chunk of conj(V_i) w.
// V_i = V + i * vstride (rhs r at r * ld); w rhs r at r * ld.  Chunk = 256 * 8 entries.
constexpr int DOT_PER_THREAD = 8;
__global__ __launch_bounds__(256) void k_dots_partial(const C64* __restrict__ V, int64_t vstride,
                                                      const C64* __restrict__ w, int64_t ld,
                                                      int64_t N, int nvec,
                                                      const int* __restrict__ active,
                                                      C64* __restrict__ partial) {
    __shared__ C64 sh[4];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int nchunk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * 256 * DOT_PER_THREAD;
    const C64* wr = w + r * ld;
    for (int ib = 0; ib < nvec; ib += 4) {
        C64 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = cx<double>(0, 0);
        for (int t = 0; t < DOT_PER_THREAD; ++t) {
            const int64_t p = base + (int64_t)t * 256 + threadIdx.x;
            if (p >= N) break;
            const C64 wp = wr[p];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (ib + q < nvec) {
                    const C64 v = V[(ib + q) * vstride + r * ld + p];
                    acc[q] = acc[q] + cjmul(v, wp);
                }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const C64 t = block_sum(acc[q], sh);
            if (threadIdx.x == 0 && ib + q < nvec)
                partial[((int64_t)r * nchunk + blockIdx.x) * nvec + ib + q] = t;
        }
    }
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// h[r * hld + i] (+)= sum over chunks of partial (fixed order: lane-strided
// sums, then a fixed butterfly).  mode 0: store, 1: add.  Also copies the
// result to hout[r * hld + i] (the coefficients of the next axpy).  One
// workgroup of four waves per right-hand side, one wave per coefficient.
__global__ __launch_bounds__(256) void k_dots_final(const C64* __restrict__ partial, int nchunk,
                                                    int nvec, const int* __restrict__ active,
                                                    C64* __restrict__ h, int hld,
                                                    C64* __restrict__ hout, int mode) {
    const int r = blockIdx.x;
    if (!active[r]) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < nvec; i += 4) {
        C64 t = cx<double>(0, 0);
        for (int c = lane; c < nchunk; c += 64) t = t + partial[((int64_t)r * nchunk + c) * nvec + i];
        t.re = wave_sum_d(t.re);
        t.im = wave_sum_d(t.im);
        if (lane == 0) {
            hout[r * hld + i] = t;
            h[r * hld + i] = mode == 0 ? t : h[r * hld + i] + t;
        }
    }
}

// w -= sum_i coef[r * cld + i] V_i  (mode 0);  x += sum_i coef V_i (mode 1).
__global__ __launch_bounds__(256) void k_axpy_multi(const C64* __restrict__ V, int64_t vstride,
                                                    C64* __restrict__ w, int64_t ld, int64_t N,
                                                    int nvec, const C64* __restrict__ coef, int cld,
                                                    const int* __restrict__ nvec_rhs,
                                                    const int* __restrict__ active, int mode) {
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= N) return;
    const int nv = nvec_rhs ? nvec_rhs[r] : nvec;
    C64 acc = cx<double>(0, 0);
    for (int i = 0; i < nv; ++i) cfma(acc, coef[r * cld + i], V[i * vstride + r * ld + p]);
    C64* wp = w + r * ld + p;
    *wp = mode == 0 ? *wp - acc : *wp + acc;
}

// The first Gram-Schmidt pass's update fused with the second pass's
// products, for a basis of NV vectors: per entry, the basis values are
// loaded once into registers, w -= sum_i coef[r * cld + i] V_i (the sum in
// the order of k_axpy_multi) is stored, and conj(V_i) w is added to the
// thread's product sums (entry by entry, as in k_dots_partial); then
// partial[(r * nchunk + chunk) * NV + i] = the workgroup's sums.  The
// results equal those of k_axpy_multi followed by k_dots_partial, with one
// read of the basis instead of two.
constexpr int AXPY_DOTS_MAXV = 16;
template <int NV>
__global__ __launch_bounds__(256) void k_axpy_dots(const C64* __restrict__ V, int64_t vstride,
                                                   C64* __restrict__ w, int64_t ld, int64_t N,
                                                   const C64* __restrict__ coef, int cld,
                                                   const int* __restrict__ active,
                                                   C64* __restrict__ partial) {
    __shared__ C64 sh[4];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int nchunk = gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * 256 * DOT_PER_THREAD;
    C64* wr = w + r * ld;
    const C64* vr = V + r * ld;
    C64 cf[NV], acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        cf[i] = coef[r * cld + i];
        acc[i] = cx<double>(0, 0);
    }
    for (int t = 0; t < DOT_PER_THREAD; ++t) {
        const int64_t p = base + (int64_t)t * 256 + threadIdx.x;
        if (p >= N) break;
        C64 v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = vr[i * vstride + p];
        C64 u = cx<double>(0, 0);
#pragma unroll
        for (int i = 0; i < NV; ++i) cfma(u, cf[i], v[i]);
        const C64 wn = wr[p] - u;
        wr[p] = wn;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = acc[i] + cjmul(v[i], wn);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const C64 t = block_sum(acc[i], sh);
        if (threadIdx.x == 0) partial[((int64_t)r * nchunk + blockIdx.x) * NV + i] = t;
    }
}

// partial[r * nchunk + chunk] = sum |w|^2 over the chunk.
__global__ __launch_bounds__(256) void k_norm_partial(const C64* __restrict__ w, int64_t ld, int64_t N,
                                                      const int* __restrict__ active,
                                                      double* __restrict__ partial) {
    __shared__ C64 sh[4];
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const int64_t base = (int64_t)blockIdx.x * 256 * DOT_PER_THREAD;
    double acc = 0;
    for (int t = 0; t < DOT_PER_THREAD; ++t) {
        const int64_t p = base + (int64_t)t * 256 + threadIdx.x;
        if (p >= N) break;
        acc += cabs2(w[r * ld + p]);
    }
    const C64 t = block_sum(cx<double>(acc, 0.0), sh);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = t.re;
}

// norm[r] = sqrt(sum of partials); if hptr: H(j+1, j) = norm.  One wave per
// right-hand side, fixed summation order.
__global__ __launch_bounds__(64) void k_norm_final(const double* __restrict__ partial, int nchunk,
                                                   const int* __restrict__ active,
                                                   double* __restrict__ norm, C64* __restrict__ hptr,
                                                   int hld) {
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    double t = 0;
    for (int c = threadIdx.x; c < nchunk; c += 64) t += partial[(int64_t)r * nchunk + c];
    t = wave_sum_d(t);
    if (threadIdx.x == 0) {
        norm[r] = sqrt(t);
        if (hptr) hptr[r * hld] = cx<double>(sqrt(t), 0.0);
    }
}

// v = w / norm[r]  (norm 0 leaves v = 0)
__global__ __launch_bounds__(256) void k_scale(const C64* __restrict__ w, C64* __restrict__ v,
                                               int64_t ld, int64_t N, const double* __restrict__ norm,
                                               const int* __restrict__ active) {
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= N) return;
    const double nr = norm[r];
    v[r * ld + p] = nr > 0 ? scale(w[r * ld + p], 1.0 / nr) : cx<double>(0, 0);
}

// Givens step j for every active right-hand side (one thread each): rotate
// column j of H by the previous rotations, form the rotation that zeroes
// H(j+1, j), update g and the relative residual estimate |g_{j+1}| / ||b||.
__global__ void k_givens(int j, int k, int nrhs, C64* __restrict__ H, double* __restrict__ cs,
                         C64* __restrict__ sn, C64* __restrict__ g, const double* __restrict__ bnorm,
                         double* __restrict__ est, const int* __restrict__ active) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs || !active[r]) return;
    C64* Hc = H + (int64_t)r * (k + 1) * k + (int64_t)j * (k + 1);
    double* c = cs + r * k;
    C64* s = sn + r * k;
    C64* gr = g + r * (k + 1);
    for (int i = 0; i < j; ++i) {
        const C64 a = Hc[i], b = Hc[i + 1];
        Hc[i] = scale(a, c[i]) + s[i] * b;
        Hc[i + 1] = scale(b, c[i]) - cx<double>(s[i].re, -s[i].im) * a;
    }
    const C64 a = Hc[j], b = Hc[j + 1];
    const double aa = sqrt(cabs2(a)), ab = sqrt(cabs2(b));
    double cj;
    C64 sj;
    if (ab == 0) {
        cj = 1.0;
        sj = cx<double>(0, 0);
    } else if (aa == 0) {
        cj = 0.0;
        sj = scale(cx<double>(b.re, -b.im), 1.0 / ab);
    } else {
        const double rr = hypot(aa, ab);
        cj = aa / rr;
        sj = scale(a, 1.0 / aa) * scale(cx<double>(b.re, -b.im), 1.0 / rr);
    }
    c[j] = cj;
    s[j] = sj;
    Hc[j] = scale(a, cj) + sj * b;
    Hc[j + 1] = cx<double>(0, 0);
    const C64 gj = gr[j];
    gr[j + 1] = -(cx<double>(sj.re, -sj.im) * gj);
    gr[j] = scale(gj, cj);
    est[r] = sqrt(cabs2(gr[j + 1])) / bnorm[r];
}

// y = R^{-1} g over the first jcount[r] Arnoldi steps (back substitution).
__global__ void k_lsq(int k, int nrhs, const C64* __restrict__ H, const C64* __restrict__ g,
                      const int* __restrict__ jcount, C64* __restrict__ y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const int jn = jcount[r];
    const C64* Hr = H + (int64_t)r * (k + 1) * k;
    for (int i = jn - 1; i >= 0; --i) {
        C64 t = g[r * (k + 1) + i];
        for (int m = i + 1; m < jn; ++m) cfms(t, Hr[(int64_t)m * (k + 1) + i], y[r * k + m]);
        y[r * k + i] = cdiv(t, Hr[(int64_t)i * (k + 1) + i]);
    }
}

// z := x over N entries of nrhs columns (column r at r * ld); nothing while
// *run is 0.
__global__ __launch_bounds__(256) void k_copy_cols(const C64* __restrict__ x, C64* __restrict__ z, int64_t ld,
                                                   int64_t N, const int* __restrict__ run) {
    if (!*run) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < N) z[blockIdx.y * ld + p] = x[blockIdx.y * ld + p];
}
void launch_copy_cols(const C64* x, C64* z, int64_t ld, int64_t N, int nrhs, const int* run, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, x, z, ld, N, run);
}

// The convergence test of GMRES on the device, after Arnoldi step j: each
// active right-hand side counts the step (iters, and jcount = the steps of
// this cycle) and leaves when its residual estimate is below rtol (a NaN
// estimate is not) or it has taken maxit steps; *run := whether any is still
// active.  One workgroup.
__global__ __launch_bounds__(256) void k_conv(int j, int nrhs, const double* __restrict__ est, double rtol,
                                              int maxit, int* __restrict__ active, int* __restrict__ iters,
                                              int* __restrict__ jcount, int* __restrict__ run) {
    if (!*run) return;
    int mine = 0;
    for (int r = threadIdx.x; r < nrhs; r += 256) {
        if (!active[r]) continue;
        const int it = iters[r] + 1;
        iters[r] = it;
        jcount[r] = j + 1;
        if (est[r] < rtol || it >= maxit)
            active[r] = 0;
        else
            mine = 1;
    }
    const int any = __syncthreads_or(mine);
    if (threadIdx.x == 0) *run = any;
}

// g = (beta, 0, ..., 0) for a new cycle.
__global__ void k_cycle_init(int k, int nrhs, const double* __restrict__ beta, C64* __restrict__ g,
                             const int* __restrict__ active) {
    const int r = blockIdx.x;
    if (r >= nrhs || !active[r]) return;
    for (int i = threadIdx.x; i <= k; i += blockDim.x)
        g[r * (k + 1) + i] = i == 0 ? cx<double>(beta[r], 0.0) : cx<double>(0, 0);
}

// ---------------------------------------------------------------------------
int dots_chunks(int64_t N) { return (int)((N + 256 * DOT_PER_THREAD - 1) / (256 * DOT_PER_THREAD)); }

void launch_dots(const C64* V, int64_t vstride, const C64* w, int64_t ld, int64_t N, int nvec,
                 int nrhs, const int* active, C64* partial, C64* h, int hld, C64* hout, int mode,
                 hipStream_t st) {
    const int nch = dots_chunks(N);
    hipLaunchKernelGGL(k_dots_partial, dim3(nch, nrhs), dim3(256), 0, st, V, vstride, w, ld, N, nvec,
                       active, partial);
    hipLaunchKernelGGL(k_dots_final, dim3(nrhs), dim3(256), 0, st, partial, nch, nvec, active, h, hld,
                       hout, mode);
}
void launch_axpy_dots(const C64* V, int64_t vstride, C64* w, int64_t ld, int64_t N, int nvec, const C64* coef,
                      int cld, int nrhs, const int* active, C64* partial, C64* h, int hld, C64* hout,
                      hipStream_t st) {
    if (nvec > AXPY_DOTS_MAXV) {  // longer bases: the two passes
        launch_axpy_multi(V, vstride, w, ld, N, nvec, coef, cld, nullptr, active, 0, nrhs, st);
        launch_dots(V, vstride, w, ld, N, nvec, nrhs, active, partial, h, hld, hout, 1, st);
        return;
    }
    const int nch = dots_chunks(N);
    const dim3 grid(nch, nrhs);
    switch (nvec) {
#define HSW_AXPY_DOTS(NV) \
    case NV: hipLaunchKernelGGL(k_axpy_dots<NV>, grid, dim3(256), 0, st, V, vstride, w, ld, N, coef, cld, active, partial); break;
        HSW_AXPY_DOTS(1) HSW_AXPY_DOTS(2) HSW_AXPY_DOTS(3) HSW_AXPY_DOTS(4) HSW_AXPY_DOTS(5) HSW_AXPY_DOTS(6)
        HSW_AXPY_DOTS(7) HSW_AXPY_DOTS(8) HSW_AXPY_DOTS(9) HSW_AXPY_DOTS(10) HSW_AXPY_DOTS(11)
        HSW_AXPY_DOTS(12) HSW_AXPY_DOTS(13) HSW_AXPY_DOTS(14) HSW_AXPY_DOTS(15) HSW_AXPY_DOTS(16)
#undef HSW_AXPY_DOTS
    default: return;  // nvec <= 0 has no products
    }
    hipLaunchKernelGGL(k_dots_final, dim3(nrhs), dim3(256), 0, st, partial, nch, nvec, active, h, hld,
                       hout, 1);
}
void launch_axpy_multi(const C64* V, int64_t vstride, C64* w, int64_t ld, int64_t N, int nvec,
                       const C64* coef, int cld, const int* nvec_rhs, const int* active, int mode,
                       int nrhs, hipStream_t st) {
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_axpy_multi, dim3(nb, nrhs), dim3(256), 0, st, V, vstride, w, ld, N, nvec, coef,
                       cld, nvec_rhs, active, mode);
}
void launch_norm(const C64* w, int64_t ld, int64_t N, int nrhs, const int* active, double* partial,
                 double* norm, C64* hptr, int hld, hipStream_t st) {
    const int nch = dots_chunks(N);
    hipLaunchKernelGGL(k_norm_partial, dim3(nch, nrhs), dim3(256), 0, st, w, ld, N, active, partial);
    hipLaunchKernelGGL(k_norm_final, dim3(nrhs), dim3(64), 0, st, partial, nch, active, norm, hptr, hld);
}
void launch_scale(const C64* w, C64* v, int64_t ld, int64_t N, int nrhs, const double* norm,
                  const int* active, hipStream_t st) {
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_scale, dim3(nb, nrhs), dim3(256), 0, st, w, v, ld, N, norm, active);
}
void launch_givens(int j, int k, int nrhs, C64* H, double* cs, C64* sn, C64* g, const double* bnorm,
                   double* est, const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_givens, dim3((nrhs + 63) / 64), dim3(64), 0, st, j, k, nrhs, H, cs, sn, g,
                       bnorm, est, active);
}
void launch_lsq(int k, int nrhs, const C64* H, const C64* g, const int* jcount, C64* y,
                hipStream_t st) {
    hipLaunchKernelGGL(k_lsq, dim3((nrhs + 63) / 64), dim3(64), 0, st, k, nrhs, H, g, jcount, y);
}
void launch_conv(int j, int nrhs, const double* est, double rtol, int maxit, int* active, int* iters,
                 int* jcount, int* run, hipStream_t st) {
    hipLaunchKernelGGL(k_conv, dim3(1), dim3(256), 0, st, j, nrhs, est, rtol, maxit, active, iters, jcount, run);
}
void launch_cycle_init(int k, int nrhs, const double* beta, C64* g, const int* active,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_cycle_init, dim3(nrhs), dim3(64), 0, st, k, nrhs, beta, g, active);
}

}  // namespace hsw
