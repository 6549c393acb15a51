// Panel solves T_i (Sec. 1.1, Alg. 1.3) on the selectively inverted fronts.
//
// A panel solve runs on an elimination-order vector of the panel's
// auxiliary box (nrhs columns, column r at r * naux):
//   gather   zero-extend the panel's planes over the artificial PML (Alg. 1.3,
//            first step; Sec. 2.3: per supernode, zero in x3) and cast to the
//            working precision;
//   forward  per depth, deepest first: each front assembles v_S from the
//            gathered values and its children's update vectors (pulled,
//            fixed order), then y = G v_S with G = [L_F^{-1}; F_BL L_F^{-1}];
//            x_S := D_F^{-1} y_S and the front's update vector is
//            w_U := (children's contributions) - y_U, i.e. the forward
//            multifrontal solve of Sec. 2.2 with L_F^{-1} applied as a product;
//   backward per depth, root first: x_S := G^T [x_S; -x_U], which equals
//            L_F^{-T}(x_S - F_BL^T x_U) (the transpose solve, applied as a product);
//   extract  scatter the panel's planes back to the padded grid and, in the
//            forward sweep, apply the coupling to the next panel (Alg. 1.5).
#include "devtypes.hpp"
#include "kernels.hpp"

namespace hsw {

// Sweep coupling J_{i+1,i} between the last plane of a panel (hi-1) and the
// next plane (hi) at lateral node (a1, a2): J[p + e3, p] = -e1 e2 ie3(hi) / h^2.
__device__ inline Cx<double> plane_coupling(const ProbDev& Q, const Cx<double>* et, int a1, int a2,
                                            int hi) {
    const Cx<double> e1 = et[Q.e_off[0] + a1];
    const Cx<double> e2 = et[Q.e_off[1] + a2];
    const Cx<double> ie3 = et[Q.e_off[2] + Q.N[2] + hi];
    return scale((e1 * e2) * ie3, -1.0 / (Q.h * Q.h));
}

// mode 0: x_in = zero extension of the panel planes of u.
// mode 1: x_in = J_{i+1,i}^T u_{i+1}: nonzero on the panel's last plane only.
// u points at plane `plane0` of the padded grid (vector r at r * ld).
template <typename T>
__global__ __launch_bounds__(256) void k_gather(int mode, ProbDev Q, PanelDev P,
                                                const int* __restrict__ perm,
                                                const Cx<double>* __restrict__ et,
                                                const Cx<double>* __restrict__ u, int64_t ld,
                                                int plane0, int nrhs, Cx<T>* __restrict__ xin,
                                                int naux) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= naux) return;
    const int NxNy = P.Nx * P.Ny;
    const int b = perm[P.perm_off + e];
    const int q = b / NxNy, lat = b - q * NxNy;
    if (mode == 0) {
        const bool live = q >= P.ga;
        const int64_t g = (int64_t)(P.lo + q - P.ga - plane0) * NxNy + lat;
        for (int r = 0; r < nrhs; ++r)
            xin[(int64_t)r * naux + e] = live ? ccast<T>(u[r * ld + g]) : cx<T>(0, 0);
    } else {
        const bool live = q == P.nz - 1;
        Cx<double> cf = cx<double>(0, 0);
        int64_t g = 0;
        if (live) {
            const int a2 = lat / P.Nx, a1 = lat - a2 * P.Nx;
            cf = plane_coupling(Q, et, a1, a2, P.hi);
            g = (int64_t)(P.hi - plane0) * NxNy + lat;
        }
        for (int r = 0; r < nrhs; ++r)
            xin[(int64_t)r * naux + e] = live ? ccast<T>(cf * u[r * ld + g]) : cx<T>(0, 0);
    }
}

// mode 0: u_i := x (panel planes), and when couple != 0 also
//         u_{i+1}(first plane) -= J_{i+1,i} u_i;  mode 1: u_i -= x.
template <typename T>
__global__ __launch_bounds__(256) void k_extract(int mode, int couple, ProbDev Q, PanelDev P,
                                                 const int* __restrict__ iperm,
                                                 const Cx<double>* __restrict__ et,
                                                 const Cx<T>* __restrict__ xout, int naux,
                                                 Cx<double>* __restrict__ u, int64_t ld, int plane0,
                                                 int nrhs) {
    const int NxNy = P.Nx * P.Ny;
    const int npanel = (P.hi - P.lo) * NxNy;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= npanel) return;
    const int pl = t / NxNy, lat = t - pl * NxNy;
    const int b = (P.ga + pl) * NxNy + lat;
    const int e = iperm[P.perm_off + b];
    const int64_t g = (int64_t)(P.lo + pl - plane0) * NxNy + lat;
    Cx<double> cf = cx<double>(0, 0);
    const bool cpl = couple && mode == 0 && (P.lo + pl == P.hi - 1);
    if (cpl) {
        const int a2 = lat / P.Nx, a1 = lat - a2 * P.Nx;
        cf = plane_coupling(Q, et, a1, a2, P.hi);
    }
    for (int r = 0; r < nrhs; ++r) {
        const Cx<double> v = ccast<double>(xout[(int64_t)r * naux + e]);
        Cx<double>* up = u + r * ld + g;
        if (mode == 0) {
            *up = v;
            if (cpl) up[NxNy] = up[NxNy] - cf * v;
        } else {
            *up = *up - v;
        }
    }
}

// Forward pass over the fronts of one depth.  Workgroup = (front, RB rows);
// the 256 threads are RB rows x 256/RB column phases.  The first eight G
// loads of every thread and the children's contributions to its update row
// are issued before the front vector is assembled, and the next eight loads
// are in flight while the current ones are consumed.  Rows of
// G_TL = L_F^{-1} above the diagonal are exact zeros, so a row block that
// lies in the triangle stops at its own last row (uniform for the workgroup).
template <typename T, int RC, int RB>
__global__ __launch_bounds__(256) void k_fwd(const int* __restrict__ work, int inst_base,
                                             const FrontInst* __restrict__ inst,
                                             const Cx<T>* __restrict__ G,
                                             const Cx<T>* __restrict__ dinv,
                                             const int* __restrict__ cmap,
                                             const Cx<T>* __restrict__ xin, Cx<T>* __restrict__ xmid,
                                             Cx<T>* __restrict__ wv, int naux, int Wld, int nrhs) {
    constexpr int P = 256 / RB;  // column phases
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    const int fcl = work[2 * blockIdx.x], rb = work[2 * blockIdx.x + 1];
    const FrontInst f = inst[inst_base + fcl];
    const int n = f.s + f.u, s = f.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, nrhs - rhs0);
    Cx<T>* vS = sm;              // [RC][s]
    Cx<T>* red = sm + RC * s;    // [P][RB][RC]
    const int tid = threadIdx.x;
    const int lr = tid % RB, ph = tid / RB;
    const int row = rb * RB + lr;
    const int kend = (rb * RB + RB <= s) ? rb * RB + RB : s;  // block-uniform
    const int rowc = row < n ? row : n - 1;  // out-of-range lanes load a valid address
    const Cx<T>* g = G + f.loff + rowc;
    Cx<T> cur[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cur[q] = g[(int64_t)min(ph + P * q, kend - 1) * n];
    const int c0i = f.child0, c1i = f.child1;
    const int* map0 = cmap + f.moff;
    const int* map1 = map0 + n;
    Cx<T> pre[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) pre[r] = cx<T>(0, 0);
    if (ph == 0 && row < n && row >= s) {
        const int p0 = c0i >= 0 ? map0[row] : -1;
        const int p1 = c1i >= 0 ? map1[row] : -1;
#pragma unroll
        for (int r = 0; r < RC; ++r)
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                if (p0 >= 0) pre[r] = pre[r] + wv[rr * Wld + f.cw0 + p0];
                if (p1 >= 0) pre[r] = pre[r] + wv[rr * Wld + f.cw1 + p1];
            }
    }
    for (int k = tid; k < s; k += 256) {
        const int p0 = c0i >= 0 ? map0[k] : -1, p1 = c1i >= 0 ? map1[k] : -1;
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            Cx<T> v = cx<T>(0, 0);
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                v = xin[rr * naux + f.start + k];
                if (p0 >= 0) v = v + wv[rr * Wld + f.cw0 + p0];
                if (p1 >= 0) v = v + wv[rr * Wld + f.cw1 + p1];
            }
            vS[r * s + k] = v;
        }
    }
    __syncthreads();
    Cx<T> acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = cx<T>(0, 0);
    for (int k = ph; k < kend; k += 8 * P) {
        const int kn = k + 8 * P;
        Cx<T> nxt[8];
        if (kn < kend) {
#pragma unroll
            for (int q = 0; q < 8; ++q) nxt[q] = g[(int64_t)min(kn + P * q, kend - 1) * n];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kq = k + P * q;
            if (kq < kend) {
#pragma unroll
                for (int r = 0; r < RC; ++r) cfma(acc[r], cur[q], vS[r * s + kq]);
            }
        }
        if (kn < kend) {
#pragma unroll
            for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
        }
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) red[(ph * RB + lr) * RC + r] = acc[r];
    __syncthreads();
    if (ph != 0 || row >= n) return;
    for (int r = 0; r < nr; ++r) {
        Cx<T> y = red[lr * RC + r];
#pragma unroll
        for (int p = 1; p < P; ++p) y = y + red[(p * RB + lr) * RC + r];
        const int64_t rr = rhs0 + r;
        if (row < s) xmid[rr * naux + f.start + row] = y * dinv[f.doff + row];
        else wv[rr * Wld + f.wvoff + (row - s)] = pre[r] - y;
    }
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Backward pass over the fronts of one depth.  Workgroup = (front, CB
// columns); wave w owns columns c0 + w + 4q (q < CB/4) and its lanes stride
// down the rows, eight loads in flight per lane (columns x unrolled rows),
// then reduce across the wave.  Rows above the block's first column are
// zeros of G_TL.
template <typename T, int RC, int CB>
__global__ __launch_bounds__(256) void k_bwd(const int* __restrict__ work, int inst_base,
                                             const FrontInst* __restrict__ inst,
                                             const Cx<T>* __restrict__ G,
                                             const int* __restrict__ ulist,
                                             const Cx<T>* __restrict__ xmid, Cx<T>* __restrict__ xout,
                                             int naux, int nrhs) {
    constexpr int CW = CB / 4;                                  // columns per wave
    constexpr int QW = CW < 8 / RC ? CW : (8 / RC > 0 ? 8 / RC : 1);  // columns per pass
    constexpr int RU = 8 / QW > 0 ? 8 / QW : 1;                 // unrolled row steps
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* rv = reinterpret_cast<Cx<T>*>(smem_raw);  // [RC][n]
    const int fcl = work[2 * blockIdx.x], cbk = work[2 * blockIdx.x + 1];
    const FrontInst f = inst[inst_base + fcl];
    const int n = f.s + f.u, s = f.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, nrhs - rhs0);
    const int tid = threadIdx.x;
    const int c0 = cbk * CB;
    const int wave = tid >> 6, lane = tid & 63;
    const Cx<T>* gb = G + f.loff;
    // first row batch of pass 0, issued before the front vector is assembled
    int cols[QW];
    bool live[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) {
        const int j = c0 + wave + 4 * q;
        live[q] = j < s;
        cols[q] = live[q] ? j : s - 1;
    }
    Cx<T> cur[RU][QW];
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int q = 0; q < QW; ++q)
            cur[u][q] = gb[(int64_t)cols[q] * n + min(c0 + lane + 64 * u, n - 1)];
    for (int i = c0 + tid; i < n; i += 256) {
        const int e = i < s ? f.start + i : ulist[f.uoff + i - s];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            Cx<T> v = cx<T>(0, 0);
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                v = i < s ? xmid[rr * naux + e] : -xout[rr * naux + e];
            }
            rv[r * n + i] = v;
        }
    }
    __syncthreads();
    for (int pass = 0; pass < CW / QW; ++pass) {
        if (pass > 0) {
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const int j = c0 + wave + 4 * (pass * QW + q);
                live[q] = j < s;
                cols[q] = live[q] ? j : s - 1;
            }
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int q = 0; q < QW; ++q)
                    cur[u][q] = gb[(int64_t)cols[q] * n + min(c0 + lane + 64 * u, n - 1)];
        }
        Cx<T> acc[QW][RC];
#pragma unroll
        for (int q = 0; q < QW; ++q)
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[q][r] = cx<T>(0, 0);
        for (int i0 = c0 + lane; i0 < n; i0 += 64 * RU) {
            const int in = i0 + 64 * RU;
            Cx<T> nxt[RU][QW];
            if (in < n) {
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int q = 0; q < QW; ++q)
                        nxt[u][q] = gb[(int64_t)cols[q] * n + min(in + 64 * u, n - 1)];
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int i = i0 + 64 * u;
                if (i < n) {
#pragma unroll
                    for (int q = 0; q < QW; ++q)
#pragma unroll
                        for (int r = 0; r < RC; ++r) cfma(acc[q][r], cur[u][q], rv[r * n + i]);
                }
            }
            if (in < n) {
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int q = 0; q < QW; ++q) cur[u][q] = nxt[u][q];
            }
        }
#pragma unroll
        for (int q = 0; q < QW; ++q)
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                acc[q][r].re = wave_sum(acc[q][r].re);
                acc[q][r].im = wave_sum(acc[q][r].im);
            }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < QW; ++q)
                if (live[q])
                    for (int r = 0; r < nr; ++r)
                        xout[(int64_t)(rhs0 + r) * naux + f.start + cols[q]] = acc[q][r];
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_gather(int mode, const ProbDev& Q, const PanelDev& P, const int* perm,
                   const Cx<double>* et, const Cx<double>* u, int64_t ld, int plane0, int nrhs,
                   Cx<T>* xin, int naux, hipStream_t st) {
    hipLaunchKernelGGL(k_gather<T>, dim3((naux + 255) / 256), dim3(256), 0, st, mode, Q, P, perm, et,
                       u, ld, plane0, nrhs, xin, naux);
}
template <typename T>
void launch_extract(int mode, int couple, const ProbDev& Q, const PanelDev& P, const int* iperm,
                    const Cx<double>* et, const Cx<T>* xout, int naux, Cx<double>* u, int64_t ld,
                    int plane0, int nrhs, hipStream_t st) {
    const int npanel = (P.hi - P.lo) * P.Nx * P.Ny;
    hipLaunchKernelGGL(k_extract<T>, dim3((npanel + 255) / 256), dim3(256), 0, st, mode, couple, Q, P,
                       iperm, et, xout, naux, u, ld, plane0, nrhs);
}

template <typename T, int RC, int RB>
static void fwd_rc(const int* work, int nwork, int inst_base, const FrontInst* inst, const Cx<T>* G,
                   const Cx<T>* dinv, const int* cmap, const Cx<T>* xin, Cx<T>* xmid, Cx<T>* wv,
                   int naux, int Wld, int nrhs, int smax, hipStream_t st) {
    size_t shm = sizeof(Cx<T>) * ((size_t)RC * smax + 256 * RC);
    dim3 grid(nwork, (nrhs + RC - 1) / RC);
    HSW_LAUNCH((k_fwd<T, RC, RB>), grid, dim3(256), shm, st, work, inst_base, inst, G, dinv, cmap,
               xin, xmid, wv, naux, Wld, nrhs);
}
template <typename T, int RC, int CB>
static void bwd_rc(const int* work, int nwork, int inst_base, const FrontInst* inst, const Cx<T>* G,
                   const int* ulist, const Cx<T>* xmid, Cx<T>* xout, int naux, int nrhs, int nmax,
                   hipStream_t st) {
    size_t shm = sizeof(Cx<T>) * (size_t)RC * nmax;
    dim3 grid(nwork, (nrhs + RC - 1) / RC);
    HSW_LAUNCH((k_bwd<T, RC, CB>), grid, dim3(256), shm, st, work, inst_base, inst, G, ulist, xmid,
               xout, naux, nrhs);
}

// Right-hand sides per workgroup: as many as fit 64 KiB of LDS (front vector
// plus the forward pass's reduction buffer), at most 8.
template <typename T>
int solve_rhs_chunk(int nrhs, int nmax) {
    int rc = 8;
    while (rc > 1 && (size_t)rc * (nmax + 256) * sizeof(Cx<T>) > 65536) rc >>= 1;
    while (rc > 1 && rc / 2 >= nrhs) rc >>= 1;
    return rc;
}

template <typename T, int RB>
static void fwd_rb(const int* work, int nwork, int inst_base, const FrontInst* inst, const Cx<T>* G,
                   const Cx<T>* dinv, const int* cmap, const Cx<T>* xin, Cx<T>* xmid, Cx<T>* wv,
                   int naux, int Wld, int nrhs, int smax, int nmax, hipStream_t st) {
    switch (solve_rhs_chunk<T>(nrhs, nmax)) {
        case 8: fwd_rc<T, 8, RB>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, st); break;
        case 4: fwd_rc<T, 4, RB>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, st); break;
        case 2: fwd_rc<T, 2, RB>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, st); break;
        default: fwd_rc<T, 1, RB>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, st); break;
    }
}
template <typename T, int CB>
static void bwd_cb(const int* work, int nwork, int inst_base, const FrontInst* inst, const Cx<T>* G,
                   const int* ulist, const Cx<T>* xmid, Cx<T>* xout, int naux, int nrhs, int nmax,
                   hipStream_t st) {
    switch (solve_rhs_chunk<T>(nrhs, nmax)) {
        case 8: bwd_rc<T, 8, CB>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st); break;
        case 4: bwd_rc<T, 4, CB>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st); break;
        case 2: bwd_rc<T, 2, CB>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st); break;
        default: bwd_rc<T, 1, CB>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st); break;
    }
}

template <typename T>
void launch_fwd(const int* work, int nwork, int rb, int inst_base, const FrontInst* inst, const Cx<T>* G,
                const Cx<T>* dinv, const int* cmap, const Cx<T>* xin, Cx<T>* xmid, Cx<T>* wv,
                int naux, int Wld, int nrhs, int smax, int nmax, hipStream_t st) {
    if (nwork <= 0) return;
    if (rb == SOLVE_RB_SMALL)
        fwd_rb<T, SOLVE_RB_SMALL>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, nmax, st);
    else
        fwd_rb<T, SOLVE_RB>(work, nwork, inst_base, inst, G, dinv, cmap, xin, xmid, wv, naux, Wld, nrhs, smax, nmax, st);
}
template <typename T>
void launch_bwd(const int* work, int nwork, int cb, int inst_base, const FrontInst* inst, const Cx<T>* G,
                const int* ulist, const Cx<T>* xmid, Cx<T>* xout, int naux, int nrhs, int nmax,
                hipStream_t st) {
    if (nwork <= 0) return;
    if (cb == SOLVE_CB_SMALL)
        bwd_cb<T, SOLVE_CB_SMALL>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st);
    else
        bwd_cb<T, SOLVE_CB>(work, nwork, inst_base, inst, G, ulist, xmid, xout, naux, nrhs, nmax, st);
}

#define HSW_INST(T)                                                                               \
    template void launch_gather<T>(int, const ProbDev&, const PanelDev&, const int*,             \
                                   const Cx<double>*, const Cx<double>*, int64_t, int, int,      \
                                   Cx<T>*, int, hipStream_t);                                    \
    template void launch_extract<T>(int, int, const ProbDev&, const PanelDev&, const int*,       \
                                    const Cx<double>*, const Cx<T>*, int, Cx<double>*, int64_t,  \
                                    int, int, hipStream_t);                                      \
    template void launch_fwd<T>(const int*, int, int, int, const FrontInst*, const Cx<T>*,       \
                                const Cx<T>*, const int*, const Cx<T>*, Cx<T>*, Cx<T>*, int, int, \
                                int, int, int, hipStream_t);                                     \
    template void launch_bwd<T>(const int*, int, int, int, const FrontInst*, const Cx<T>*,       \
                                const int*,                                                      \
                                const Cx<T>*, Cx<T>*, int, int, int, hipStream_t);               \
    template int solve_rhs_chunk<T>(int, int);
HSW_INST(float)
HSW_INST(double)
#undef HSW_INST

}  // namespace hsw
