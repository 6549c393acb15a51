// Batched multifrontal partial LDL^T of the panels' auxiliary problems
// (Sec. 2.2) and the selectively inverted fronts used by the solves.
//
// Every launch covers all fronts of one elimination-tree depth over all
// panels and problems; a flat work list of (front instance, tile or block)
// pairs maps workgroups to work, so fronts of uneven size share a launch.
//
// Front storage.  A front with s pivots and u update rows is the
// (s+u) x (s+u) lower triangle F = [F_TL *; F_BL F_BR].  Its first s columns
// [F_TL; F_BL] live in the persistent factor buffer as an (s+u) x s
// column-major block (leading dimension s+u); F_BR (u x u, column-major)
// lives in a workspace indexed by the parity of the depth, kept until the
// parent has pulled it (extend-add) one level up.
#include "devtypes.hpp"
#include "kernels.hpp"
#include "stencil.hpp"

namespace hsw {

__device__ inline void tri_decode_dev(int t, int& ti, int& tj) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
}

template <typename T>
__device__ inline Cx<T>* front_at(Cx<T>* L, Cx<T>* W, int n, int s, int u, int i, int j) {
    return j < s ? L + (int64_t)j * n + i : W + (int64_t)(j - s) * u + (i - s);
}

// Entry H(bi, bj) of a panel's auxiliary operator between box nodes bi, bj
// (box index a1 + a2 Nx + q Nx Ny); zero when they are not stencil neighbours.
__device__ inline Cx<double> aux_entry(const ProbDev& Q, const PanelDev& P, const Cx<double>* et,
                                       int bi, int bj, Cx<double> kappa2, double inv_h2) {
    const int NxNy = P.Nx * P.Ny;
    int qi = bi / NxNy, ri = bi - qi * NxNy, a2i = ri / P.Nx, a1i = ri - a2i * P.Nx;
    int qj = bj / NxNy, rj = bj - qj * NxNy, a2j = rj / P.Nx, a1j = rj - a2j * P.Nx;
    const Cx<double>* e3n = et + P.e3_off;
    const Cx<double>* ie3 = et + P.e3_off + P.nz;
    if (bi == bj) {
        NodeStretch st = node_stretch(Q, et, a1i, a2i, e3n, ie3, qi);
        double c = velocity_at(Q, a1i, a2i, P.lo - P.ga + qi);
        return diag_entry(st, c, kappa2, inv_h2);
    }
    int d1 = a1i - a1j, d2 = a2i - a2j, d3 = qi - qj;
    int ad = abs(d1) + abs(d2) + abs(d3);
    if (ad != 1) return cx<double>(0.0, 0.0);
    int ax = d1 != 0 ? 0 : (d2 != 0 ? 1 : 2);
    int sgn = d1 + d2 + d3;  // +1: i is the upper node
    int la1 = sgn > 0 ? a1j : a1i, la2 = sgn > 0 ? a2j : a2i, lq = sgn > 0 ? qj : qi;
    NodeStretch st = node_stretch(Q, et, la1, la2, e3n, ie3, lq);
    return upper_coupling(st, ax, inv_h2);
}

// ---------------------------------------------------------------------------
// Front assembly: original entries of H_i in the pivot columns plus the
// extend-add of the children's update matrices (pulled, fixed order: no
// atomics, bitwise deterministic).  One workgroup per 64 x 64 lower tile.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const int2* __restrict__ work,
                                                  const FrontInst* __restrict__ inst,
                                                  const PanelDev* __restrict__ pan,
                                                  const ProbDev* __restrict__ prob,
                                                  const int* __restrict__ perm,
                                                  const int* __restrict__ ulist,
                                                  const int* __restrict__ cmap,
                                                  const Cx<double>* __restrict__ et,
                                                  Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ Wcur,
                                                  const Cx<T>* __restrict__ Wchild) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    int ti, tj;
    tri_decode_dev(w.y, ti, tj);
    const int r0 = ti * TILE, c0 = tj * TILE;
    __shared__ int rpos[2][TILE], cpos[2][TILE], rbox[TILE], cbox[TILE];
    const int tid = threadIdx.x;
    const PanelDev P = pan[f.panel];
    if (tid < 2 * TILE) {
        const bool isrow = tid < TILE;
        const int l = isrow ? tid : tid - TILE;
        const int i = (isrow ? r0 : c0) + l;
        int bx = -1, p0 = -1, p1 = -1;
        if (i < n) {
            int e = i < f.s ? f.start + i : ulist[f.uoff + i - f.s];
            bx = perm[P.perm_off + e];
            if (f.child0 >= 0) p0 = cmap[f.moff + i];
            if (f.child1 >= 0) p1 = cmap[f.moff + n + i];
        }
        if (isrow) { rbox[l] = bx; rpos[0][l] = p0; rpos[1][l] = p1; }
        else { cbox[l] = bx; cpos[0][l] = p0; cpos[1][l] = p1; }
    }
    __syncthreads();
    const ProbDev Q = prob[P.prob];
    const Cx<double> kappa2 = kappa_sq(Q, Q.alpha);
    const double inv_h2 = 1.0 / (Q.h * Q.h);
    int64_t cw[2] = {0, 0};
    int cu[2] = {0, 0};
    if (f.child0 >= 0) { cw[0] = inst[f.child0].woff; cu[0] = inst[f.child0].u; }
    if (f.child1 >= 0) { cw[1] = inst[f.child1].woff; cu[1] = inst[f.child1].u; }
    Cx<T>* L = Lb + f.loff;
    Cx<T>* W = Wcur + f.woff;
    for (int idx = tid; idx < TILE * TILE; idx += 256) {
        const int li = idx & (TILE - 1), lj = idx / TILE;
        const int i = r0 + li, j = c0 + lj;
        if (i >= n || j >= n || i < j) continue;
        Cx<T> acc = cx<T>(0, 0);
        if (j < f.s) acc = ccast<T>(aux_entry(Q, P, et, rbox[li], cbox[lj], kappa2, inv_h2));
        for (int ch = 0; ch < 2; ++ch) {
            int pi = rpos[ch][li], pj = cpos[ch][lj];
            if (pi >= 0 && pj >= 0) acc = acc + Wchild[cw[ch] + (int64_t)pj * cu[ch] + pi];
        }
        *front_at(L, W, n, f.s, f.u, i, j) = acc;
    }
}

// ---------------------------------------------------------------------------
// Diagonal block [k, k+b) of the blocked partial LDL^T: one workgroup per
// front factors the b x b block in LDS (unpivoted, transposes only) and
// writes L_kk (unit lower, below the diagonal), the pivots D_kk (on the
// diagonal) and their reciprocals.  A zero or non-finite pivot is reported.
template <typename T>
__global__ __launch_bounds__(256) void k_ldlt_diag(const int2* __restrict__ work,
                                                   const FrontInst* __restrict__ inst,
                                                   Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ dinv,
                                                   int k, int* __restrict__ err) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    const int b = min(NB, f.s - k);
    Cx<T>* L = Lb + f.loff;
    __shared__ Cx<T> A[NB][NB + 1];  // A[col][row]
    __shared__ Cx<T> dv[NB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = -1;
    for (int idx = tid; idx < NB * NB; idx += 256) {
        int row = idx & (NB - 1), col = idx / NB;
        if (row < b && col < b && row >= col) A[col][row] = L[(int64_t)(k + col) * n + k + row];
    }
    __syncthreads();
    for (int m = 0; m < b; ++m) {
        const Cx<T> dm = A[m][m];
        const Cx<T> idm = crecip(dm);
        const int jj = tid & 63;
        if (jj > m && jj < b) {
            const Cx<T> ljj = A[m][jj] * idm;
            for (int i = jj + (tid >> 6); i < b; i += 4) cfms(A[jj][i], A[m][i], ljj);
        }
        if (tid == 0) {
            dv[m] = idm;
            bool finite = isfinite(dm.re) && isfinite(dm.im) && isfinite(idm.re) && isfinite(idm.im);
            if (!finite || (dm.re == 0 && dm.im == 0)) { if (bad < 0) bad = m; }
        }
        __syncthreads();
        if (tid > m && tid < b) A[m][tid] = A[m][tid] * idm;
        __syncthreads();
    }
    for (int idx = tid; idx < NB * NB; idx += 256) {
        int row = idx & (NB - 1), col = idx / NB;
        if (row < b && col < b && row >= col) L[(int64_t)(k + col) * n + k + row] = A[col][row];
    }
    if (tid < b) dinv[f.doff + k + tid] = dv[tid];
    if (tid == 0 && bad >= 0) {
        if (atomicCAS(&err[0], -1, w.x) == -1) err[1] = k + bad;
    }
}

// Panel rows below the diagonal block: F_BL := F_BL L_kk^{-T} D_kk^{-1} for 64
// rows per workgroup, reading the already factored diagonal block.
template <typename T>
__global__ __launch_bounds__(256) void k_panel_trsm(const int2* __restrict__ work,
                                                    const FrontInst* __restrict__ inst,
                                                    Cx<T>* __restrict__ Lb,
                                                    const Cx<T>* __restrict__ dinv, int k) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    const int b = min(NB, f.s - k);
    Cx<T>* L = Lb + f.loff;
    __shared__ Cx<T> Lk[NB][NB + 1];  // Lk[m][jj] = L_kk(jj, m), jj > m
    __shared__ Cx<T> Pn[NB][NB + 1];  // panel rows, Pn[col][row]
    __shared__ Cx<T> dv[NB];
    const int tid = threadIdx.x;
    const int rbeg = k + b + w.y * 64, rend = min(rbeg + 64, n);
    for (int idx = tid; idx < NB * NB; idx += 256) {
        int row = idx & (NB - 1), col = idx / NB;
        if (row < b && col < b && row > col) Lk[col][row] = L[(int64_t)(k + col) * n + k + row];
        int r = rbeg + row;
        if (col < b && r < rend) Pn[col][row] = L[(int64_t)(k + col) * n + r];
    }
    if (tid < b) dv[tid] = dinv[f.doff + k + tid];
    __syncthreads();
    const int lr = tid & 63, jg = tid >> 6;
    const bool active = rbeg + lr < rend;
    for (int m = 0; m < b; ++m) {
        if (active) {
            const Cx<T> y = Pn[m][lr];
            for (int jj = jg; jj < b; jj += 4)
                if (jj > m) cfms(Pn[jj][lr], y, Lk[m][jj]);
        }
        __syncthreads();
    }
    if (active)
        for (int col = jg; col < b; col += 4)
            L[(int64_t)(k + col) * n + rbeg + lr] = Pn[col][lr] * dv[col];
}

// ---------------------------------------------------------------------------
// Trailing update of pivot block [k, k+b): F[i,j] -= sum_m X[i,m] d_m X[j,m]
// over the lower triangle of rows/columns [k+b, s+u) -- the F_BR := F_BR -
// Z F_BL^T Schur update of Sec. 2.2 applied blockwise, plus the update of
// the remaining pivot columns.  One workgroup per 64 x 64 output tile.
template <typename T>
__global__ __launch_bounds__(256) void k_trailing(const int2* __restrict__ work,
                                                  const FrontInst* __restrict__ inst,
                                                  Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ Wcur,
                                                  int k) {
    constexpr int KC = 16;
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    const int b = min(NB, f.s - k);
    const int t0 = k + b;
    int ti, tj;
    tri_decode_dev(w.y, ti, tj);
    const int r0 = t0 + ti * TILE, c0 = t0 + tj * TILE;
    Cx<T>* L = Lb + f.loff;
    Cx<T>* W = Wcur + f.woff;
    __shared__ Cx<T> Xr[KC][TILE], Xc[KC][TILE];
    __shared__ Cx<T> dd[NB];
    const int tid = threadIdx.x;
    if (tid < b) dd[tid] = L[(int64_t)(k + tid) * n + k + tid];
    const int lr = tid & 63, cb = (tid >> 6) * 16;
    Cx<T> acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = cx<T>(0, 0);
    __syncthreads();
    for (int kc = 0; kc < b; kc += KC) {
        for (int idx = tid; idx < KC * TILE; idx += 256) {
            int l = idx & 63, m = idx / 64;
            int km = kc + m;
            Cx<T> xr = cx<T>(0, 0), xc = cx<T>(0, 0);
            if (km < b) {
                const Cx<T>* col = L + (int64_t)(k + km) * n;
                if (r0 + l < n) xr = col[r0 + l];
                if (c0 + l < n) xc = col[c0 + l] * dd[km];
            }
            Xr[m][l] = xr;
            Xc[m][l] = xc;
        }
        __syncthreads();
#pragma unroll 4
        for (int m = 0; m < KC; ++m) {
            const Cx<T> x = Xr[m][lr];
#pragma unroll
            for (int c = 0; c < 16; ++c) cfma(acc[c], x, Xc[m][cb + c]);
        }
        __syncthreads();
    }
    const int i = r0 + lr;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int j = c0 + cb + c;
        if (j < n && i >= j) {
            Cx<T>* p = front_at(L, W, n, f.s, f.u, i, j);
            *p = *p - acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Selective inversion (Sec. 2.2): G = X with X L_F = [I; F_BL], i.e.
// G = [L_F^{-1}; F_BL L_F^{-1}], so that both multifrontal triangular solves
// of a front become one product with G.  Rows are independent: one
// workgroup per 64 rows, sweeping the pivot columns from last to first.
template <typename T>
__global__ __launch_bounds__(256) void k_inverse(const int2* __restrict__ work,
                                                 const FrontInst* __restrict__ inst,
                                                 const Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ Gb) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u, s = f.s;
    const Cx<T>* L = Lb + f.loff;
    Cx<T>* G = Gb + f.loff;
    const int r0 = w.y * 64;
    const int tid = threadIdx.x, lr = tid & 63, cg = tid >> 6;
    const int row = r0 + lr;
    __shared__ Cx<T> Xs[64][65];  // X chunk [m][row], reused as the block accumulator [jj][row]
    __shared__ Cx<T> Ls[64][65];  // L chunk [jj][m]
    const int ncb = (s + 63) / 64;
    for (int cbk = ncb - 1; cbk >= 0; --cbk) {
        const int c0 = cbk * 64, c1 = min(c0 + 64, s), bw = c1 - c0;
        // rows of the identity above the block are zero in L_F^{-1}
        if (r0 + 63 < c0) {
            for (int jj = cg; jj < bw; jj += 4)
                if (row < n) G[(int64_t)(c0 + jj) * n + row] = cx<T>(0, 0);
            continue;
        }
        Cx<T> acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int jj = cg * 16 + q;
            Cx<T> v = cx<T>(0, 0);
            if (row < n && jj < bw) {
                if (row < s) v = cx<T>(row == c0 + jj ? (T)1 : (T)0, 0);
                else v = L[(int64_t)(c0 + jj) * n + row];
            }
            acc[q] = v;
        }
        for (int mc = c1; mc < s; mc += 64) {
            const int mw = min(64, s - mc);
            __syncthreads();
            for (int idx = tid; idx < 64 * 64; idx += 256) {
                int a = idx & 63, bq = idx / 64;
                Xs[bq][a] = (bq < mw && r0 + a < n) ? G[(int64_t)(mc + bq) * n + r0 + a] : cx<T>(0, 0);
                Ls[bq][a] = (bq < bw && a < mw) ? L[(int64_t)(c0 + bq) * n + mc + a] : cx<T>(0, 0);
            }
            __syncthreads();
            for (int m = 0; m < mw; ++m) {
                const Cx<T> x = Xs[m][lr];
#pragma unroll
                for (int q = 0; q < 16; ++q) cfms(acc[q], x, Ls[cg * 16 + q][m]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) Xs[cg * 16 + q][lr] = acc[q];
        for (int idx = tid; idx < 64 * 64; idx += 256) {
            int a = idx & 63, bq = idx / 64;  // Ls[bq][a] = L[c0 + a][c0 + bq]
            Ls[bq][a] = (bq < bw && a < bw && a > bq) ? L[(int64_t)(c0 + bq) * n + c0 + a] : cx<T>(0, 0);
        }
        __syncthreads();
        for (int jj = bw - 1; jj > 0; --jj) {
            const Cx<T> x = Xs[jj][lr];
            for (int j2 = cg; j2 < jj; j2 += 4) cfms(Xs[j2][lr], x, Ls[j2][jj]);
            __syncthreads();
        }
        if (row < n)
            for (int jj = cg; jj < bw; jj += 4) G[(int64_t)(c0 + jj) * n + row] = Xs[jj][lr];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_assemble(const int2* work, int nwork, const FrontInst* inst, const PanelDev* pan,
                     const ProbDev* prob, const int* perm, const int* ulist, const int* cmap,
                     const Cx<double>* et, Cx<T>* Lb, Cx<T>* Wcur, const Cx<T>* Wchild,
                     hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_assemble<T>, dim3(nwork), dim3(256), 0, st, work, inst, pan, prob, perm,
                       ulist, cmap, et, Lb, Wcur, Wchild);
}
template <typename T>
void launch_ldlt_diag(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* dinv,
                      int k, int* err, hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_ldlt_diag<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, dinv, k, err);
}
template <typename T>
void launch_panel_trsm(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb,
                       const Cx<T>* dinv, int k, hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_panel_trsm<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, dinv, k);
}
template <typename T>
void launch_trailing(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* Wcur,
                     int k, hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_trailing<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, Wcur, k);
}
template <typename T>
void launch_inverse(const int2* work, int nwork, const FrontInst* inst, const Cx<T>* Lb, Cx<T>* Gb,
                    hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_inverse<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, Gb);
}

#define HSW_INST(T)                                                                              \
    template void launch_assemble<T>(const int2*, int, const FrontInst*, const PanelDev*,       \
                                     const ProbDev*, const int*, const int*, const int*,        \
                                     const Cx<double>*, Cx<T>*, Cx<T>*, const Cx<T>*,           \
                                     hipStream_t);                                              \
    template void launch_ldlt_diag<T>(const int2*, int, const FrontInst*, Cx<T>*, Cx<T>*, int,   \
                                      int*, hipStream_t);                                       \
    template void launch_panel_trsm<T>(const int2*, int, const FrontInst*, Cx<T>*, const Cx<T>*, \
                                       int, hipStream_t);                                       \
    template void launch_trailing<T>(const int2*, int, const FrontInst*, Cx<T>*, Cx<T>*, int,    \
                                     hipStream_t);                                              \
    template void launch_inverse<T>(const int2*, int, const FrontInst*, const Cx<T>*, Cx<T>*,    \
                                    hipStream_t);
HSW_INST(float)
HSW_INST(double)
#undef HSW_INST

}  // namespace hsw
