// Panel solves T_i (Sec. 1.1, Alg. 1.3) on the selectively inverted fronts.
//
// A panel solve is one forward pass per tree depth, deepest first, then one
// backward pass per depth, root first:
//   forward  each front assembles v_S from the panel's right-hand side and
//            its children's contributions, then y = G v_S with
//            G = [L_F^{-1}; F_BL L_F^{-1}]; x_S := D_F^{-1} y_S, and the update
//            part (children's contributions minus y_U) goes to the front's
//            slot in its parent -- the forward multifrontal solve of Sec. 2.2
//            with L_F^{-1} applied as a product.  At the deepest fronts the
//            right-hand side is read straight from the padded grid: zero
//            extension over the artificial PML (Alg. 1.3) or the coupling
//            J_{i+1,i}^T of the next plane (Alg. 1.5), cast to the working
//            precision;
//   backward x_S := G^T [x_S; -x_U], which equals L_F^{-T}(x_S - F_BL^T x_U);
//            x_S is written to the panel's planes of the padded grid (stored
//            or subtracted, plus the coupling into the next panel of the
//            forward sweep) and pushed to the children's update-set values.
// Parents and children exchange values through slots laid out in the
// receiver's order, so no pass reads through an index it has to load first.
#include <type_traits>

#include "devtypes.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace hsw {

// J[p + e3, p] = -e1 e2 ie3(hi) / h^2 between the last plane of a panel and
// the next plane, at lateral node (a1, a2).
template <typename T>
__device__ inline Cx<double> plane_coupling(const PassArgs<T>& A, int lat) {
    const int a2 = lat / A.Nx, a1 = lat - a2 * A.Nx;
    const Cx<double> c = (A.et[A.e1 + a1] * A.et[A.e2 + a2]) * A.et[A.ie3hi];
    return scale(c, -A.inv_h2);
}

// Box index (a1 + a2 Nx + q Nx Ny) of pivot e of a front from its cell rectangle.
__device__ inline int pivot_box(const SolveItem& it, int Nx, int NxNy, int e) {
    const int x0 = it.cell0 & 0xffff, y0 = it.cell0 >> 16;
    const int cw = it.cellw & 0xffff, nc = it.cellw >> 16;
    const int q = e / nc, cell = e - q * nc;
    const int r = cell / cw;
    return x0 + (cell - r * cw) + (y0 + r) * Nx + q * NxNy;
}

template <typename T>
__device__ inline Cx<T> keep(bool on, Cx<T> v) {
    return cx<T>(on ? v.re : (T)0, on ? v.im : (T)0);
}

// Pivots of a front are ordered plane by plane (pivot e on auxiliary plane
// e / cells).  A leaf front has no children, so its forward-pass vector is
// the right-hand side alone: zero on the ga auxiliary PML planes in mode 0
// (the zero extension of the panel) and zero below the last plane in mode 1
// (the coupling J_{i+1,i}^T reaches the last plane only).  Returns the first
// pivot that can hold a non-zero entry; the product skips the columns before
// it, which multiply exact zeros.
template <typename T>
__device__ inline int leaf_first_live(const PassArgs<T>& A, const SolveItem& it) {
    if (!it.leaf) return 0;
    return (A.mode == 0 ? A.ga : A.nz - 1) * (it.cellw >> 16);
}
// The backward pass of a leaf writes only the pivots on the panel's own
// planes (the auxiliary ones are neither extracted nor needed by children):
// true when columns [c0, c0 + cb) all lie on auxiliary planes.
__device__ inline bool leaf_aux_block(const SolveItem& it, int ga, int c0, int cb) {
    return it.leaf && c0 + cb <= ga * (it.cellw >> 16);
}
// The pivots of a leaf on auxiliary planes (0 for other fronts).  In the
// matrix-core passes their x_S (exact zeros in the forward pass: zero
// right-hand side, no children) is neither stored nor read: the backward
// pass of a leaf starts its contraction at the first pivot past them, since
// the rows it skips meet only columns the upper triangle of L_F^{-1} zeros
// or columns whose results are not kept.
__device__ inline int leaf_aux_rows(const SolveItem& it, int ga) {
    return it.leaf ? ga * (it.cellw >> 16) : 0;
}

// Loads in flight per thread: the G entries a thread consumes are issued in
// rounds of QL before the previous round is used.
template <typename T> struct PassLoads { static constexpr int QL = 8; };
template <> struct PassLoads<double> { static constexpr int QL = 8; };
static_assert((PassLoads<float>::QL & (PassLoads<float>::QL - 1)) == 0 &&
                  (PassLoads<double>::QL & (PassLoads<double>::QL - 1)) == 0,
              "loads per round must be a power of two (the backward passes split a wave's "
              "power-of-two column count into rounds)");

// Forward pass over the fronts of one depth.  Workgroup = (front, RB rows),
// NT threads as RB rows x NT/RB column phases.  Rows of G_TL = L_F^{-1}
// above the diagonal are exact zeros, so a row block inside the triangle
// stops at its own last row (uniform for the workgroup).
template <typename T, int RC, int RB, int NT>
__global__ __launch_bounds__(NT) void k_fwd(PassArgs<T> A) {
    constexpr int P = NT / RB;
    constexpr int QL = PassLoads<T>::QL;
    static_assert(RB >= 1 && RB <= 64 && 64 % RB == 0 && NT % 64 == 0,
                  "a row block lies inside one wave: the phases of a row are reduced by "
                  "shuffles within the wave, then one partial per wave");
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* sm = reinterpret_cast<Cx<T>*>(smem_raw);
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    const int n = it.n, s = it.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, A.nrhs - rhs0);
    Cx<T>* vS = sm;            // [RC][s]
    Cx<T>* red = sm + RC * s;  // [waves][RB][RC]
    const int tid = threadIdx.x;
    const int lr = tid % RB, ph = tid / RB;
    const int row = it.blk + lr;
    const int kend = (it.blk + RB <= s) ? it.blk + RB : s;
    const int k0 = leaf_first_live(A, it);
    const Cx<T>* g = A.G + it.loff + min(row, n - 1);
    Cx<T> cur[QL];
#pragma unroll
    for (int q = 0; q < QL; ++q) cur[q] = cx<T>(0, 0);
    if (k0 < kend) {
#pragma unroll
        for (int q = 0; q < QL; ++q) cur[q] = g[(int64_t)min(k0 + ph + P * q, kend - 1) * n];
    }
    const int* map0 = A.cmap + it.moff;
    const int* map1 = map0 + n;
    // the output row's operands (threads of phase 0)
    Cx<T> pre[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) pre[r] = cx<T>(0, 0);
    Cx<T> dv = cx<T>(0, 0);
    int pm = 0;
    if (ph == 0 && row < n) {
        if (row < s) {
            dv = A.dinv[it.start + row];
        } else {
            pm = A.pmap[it.pmap + row - s];
            const bool h0 = map0[row] >= 0, h1 = map1[row] >= 0;
#pragma unroll
            for (int r = 0; r < RC; ++r)
                if (r < nr) {
                    const Cx<T>* cc = A.c2 + (int64_t)(rhs0 + r) * A.c2ld + it.c2;
                    const Cx<T> a0 = cc[row], a1 = cc[n + row];
                    pre[r] = keep(h0, a0) + keep(h1, a1);
                }
        }
    }
    // front vector: right-hand side on the panel plus the children's slots;
    // slots a child does not cover hold stale values and are masked out
    for (int k = k0 + tid; k < s; k += NT) {
        const int b = pivot_box(it, A.Nx, A.NxNy, k);
        const int q = b / A.NxNy, lat = b - q * A.NxNy;
        const bool h0 = map0[k] >= 0, h1 = map1[k] >= 0;
        bool live;
        int64_t gi;
        Cx<double> cf = cx<double>(1, 0);
        if (A.mode == 0) {
            live = q >= A.ga;
            gi = (int64_t)(A.lo + q - A.ga - A.plane0) * A.NxNy + lat;
        } else {
            live = q == A.nz - 1;
            gi = (int64_t)(A.hi - A.plane0) * A.NxNy + lat;
            if (live) cf = plane_coupling(A, lat);
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            Cx<T> v = cx<T>(0, 0);
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                const Cx<T>* cc = A.c2 + rr * A.c2ld + it.c2;
                const Cx<T> a0 = cc[k], a1 = cc[n + k];
                v = keep(h0, a0) + keep(h1, a1);
                if (live) {
                    const Cx<double> x = A.src[rr * A.ld + gi];
                    v = v + ccast<T>(A.mode == 0 ? x : cf * x);
                }
            }
            vS[r * s + k] = v;
        }
    }
    __syncthreads();
    Cx<T> acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = cx<T>(0, 0);
    for (int k = k0 + ph; k < kend; k += QL * P) {
        const int kn = k + QL * P;
        Cx<T> nxt[QL];
        if (kn < kend) {
#pragma unroll
            for (int q = 0; q < QL; ++q) nxt[q] = g[(int64_t)min(kn + P * q, kend - 1) * n];
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const int kq = k + P * q;
            if (kq < kend) {
#pragma unroll
                for (int r = 0; r < RC; ++r) cfma(acc[r], cur[q], vS[r * s + kq]);
            }
        }
        if (kn < kend) {
#pragma unroll
            for (int q = 0; q < QL; ++q) cur[q] = nxt[q];
        }
    }
    // reduce the phases: inside the wave by shuffles, then across waves
#pragma unroll
    for (int r = 0; r < RC; ++r)
#pragma unroll
        for (int off = RB; off < 64; off <<= 1) {
            acc[r].re += __shfl_xor(acc[r].re, off, 64);
            acc[r].im += __shfl_xor(acc[r].im, off, 64);
        }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane < RB) {
#pragma unroll
        for (int r = 0; r < RC; ++r) red[(wave * RB + lane) * RC + r] = acc[r];
    }
    __syncthreads();
    if (tid >= RB || row >= n) return;  // tid < RB: phase 0, lr == tid
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        if (r >= nr) break;
        Cx<T> y = red[lr * RC + r];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) y = y + red[(w * RB + lr) * RC + r];
        const int64_t rr = rhs0 + r;
        if (row < s) A.xmid[rr * A.naux + it.start + row] = y * dv;
        else A.c2[rr * A.c2ld + it.push + pm] = pre[r] - y;
    }
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Backward pass over the fronts of one depth.  Workgroup = (front, CB
// columns, NT threads); wave w of the NW = NT/64 waves owns columns
// c0 + w + NW q (q < CB/NW) and its lanes stride
// down the rows with QL loads in flight, then reduce across the wave.  Rows
// above the block's first column are zeros of G_TL.
template <typename T, int RC, int CB, int NT>
__global__ __launch_bounds__(NT) void k_bwd(PassArgs<T> A) {
    constexpr int NW = NT / 64;
    constexpr int QL = PassLoads<T>::QL;
    constexpr int CW = CB / NW;                                    // columns per wave
    constexpr int QW = CW < QL / RC ? CW : (QL / RC > 0 ? QL / RC : 1);  // columns per pass
    constexpr int RU = QL / QW > 0 ? QL / QW : 1;                  // unrolled row steps
    static_assert(CW >= 1 && CW <= 64, "column block");
    static_assert(CW % QW == 0, "the passes must cover every column of the wave");
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* rv = reinterpret_cast<Cx<T>*>(smem_raw);  // [RC][n]
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    if (leaf_aux_block(it, A.ga, it.blk, CB)) return;
    const int n = it.n, s = it.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, A.nrhs - rhs0);
    const int tid = threadIdx.x;
    const int c0 = it.blk;
    const int wave = tid >> 6, lane = tid & 63;
    const Cx<T>* gb = A.G + it.loff;
    int cols[QW];
    bool live[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) {
        const int j = c0 + wave + NW * q;
        live[q] = j < s;
        cols[q] = live[q] ? j : s - 1;
    }
    Cx<T> cur[RU][QW];
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int q = 0; q < QW; ++q)
            cur[u][q] = gb[(int64_t)cols[q] * n + min(c0 + lane + 64 * u, n - 1)];
    // lane l < CW of each wave owns the output of the wave's column l
    const int jl = c0 + wave + NW * lane;
    const bool own = lane < CW && jl < s;
    int o0 = -1, o1 = -1;
    int64_t ogi = 0;
    bool oplane = false, onext = false;
    Cx<double> ocf = cx<double>(0, 0);
    if (own) {
        const int b = pivot_box(it, A.Nx, A.NxNy, jl);
        const int q = b / A.NxNy, lat = b - q * A.NxNy;
        oplane = q >= A.ga;
        ogi = (int64_t)(A.lo + q - A.ga - A.plane0) * A.NxNy + lat;
        onext = A.couple && A.mode == 0 && q == A.nz - 1;
        if (onext) ocf = plane_coupling(A, lat);
        if (it.cxu0 >= 0) o0 = A.cmap[it.moff + jl];
        if (it.cxu1 >= 0) o1 = A.cmap[it.moff + n + jl];
    }
    // the padded grid's old values the epilogue updates (mode 1: the pivot's
    // own entry; mode 0 with the coupling: the next plane's), read now so
    // that they arrive during the products
    Cx<double> oold[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        oold[r] = cx<double>(0, 0);
        if (own && oplane && r < nr && (A.mode != 0 || onext))
            oold[r] = A.dst[(rhs0 + r) * A.ld + ogi + (A.mode != 0 ? 0 : A.NxNy)];
    }
    // [x_S; -x_U] of this front (loads only: nothing in this loop waits on a
    // loaded value before the next load)
    for (int i = c0 + tid; i < n; i += NT) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            Cx<T> v = cx<T>(0, 0);
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                v = i < s ? A.xmid[rr * A.naux + it.start + i] : -A.xu[rr * A.xuld + it.xu + i - s];
            }
            rv[r * n + i] = v;
        }
    }
    // The update-set values go on to the children.  The front's column
    // blocks share its u rows, and each thread issues the loads of four rows
    // before their stores, so the map lookups do not form one long chain of
    // memory round trips.
    if (it.cxu0 >= 0 || it.cxu1 >= 0) {
        const int u = n - s;
        const int nb = (s + CB - 1) / CB, b = c0 / CB;
        const int per = (u + nb - 1) / nb;
        const int i_lo = s + b * per, i_hi = min(n, i_lo + per);
        for (int i0 = i_lo + tid; i0 < i_hi; i0 += 4 * NT) {
            Cx<T> xv[4][RC];
            int p0[4], p1[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * NT;
                const bool ok = i < i_hi;
                p0[k] = ok && it.cxu0 >= 0 ? A.cmap[it.moff + i] : -1;
                p1[k] = ok && it.cxu1 >= 0 ? A.cmap[it.moff + n + i] : -1;
#pragma unroll
                for (int r = 0; r < RC; ++r)
                    xv[k][r] = ok && r < nr ? A.xu[(rhs0 + r) * A.xuld + it.xu + i - s] : cx<T>(0, 0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int r = 0; r < RC; ++r) {
                    if (r >= nr) break;
                    const int64_t rr = rhs0 + r;
                    if (p0[k] >= 0) A.xu[rr * A.xuld + it.cxu0 + p0[k]] = xv[k][r];
                    if (p1[k] >= 0) A.xu[rr * A.xuld + it.cxu1 + p1[k]] = xv[k][r];
                }
        }
    }
    __syncthreads();
    for (int pass = 0; pass < CW / QW; ++pass) {
        if (pass > 0) {
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const int j = c0 + wave + NW * (pass * QW + q);
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
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            if (!own || lane != pass * QW + q) continue;
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                if (r >= nr) break;
                const int64_t rr = rhs0 + r;
                const Cx<T> x = acc[q][r];
                if (o0 >= 0) A.xu[rr * A.xuld + it.cxu0 + o0] = x;
                if (o1 >= 0) A.xu[rr * A.xuld + it.cxu1 + o1] = x;
                if (oplane) {
                    Cx<double>* up = A.dst + rr * A.ld + ogi;
                    const Cx<double> xd = ccast<double>(x);
                    if (A.mode == 0) {
                        *up = xd;
                        if (onext) up[A.NxNy] = oold[r] - ocf * xd;
                    } else {
                        *up = oold[r] - xd;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Passes for groups of 16 right-hand sides on the matrix cores: the products
// G v_S and G^T [x_S; -x_U] of the panel solves become GEMMs with 16 columns
// (the sweeps of many sources applied at once).  Every vector of these passes
// is held as [entry][16] blocks (the 16 right-hand sides of an entry
// contiguous, one block of entries per group), so each operand chunk is a
// dense, coalesced read:
//   * at the start of a panel solve the scatter puts the panel's right-hand
//     side, in elimination order, into h2 (zero extension over the auxiliary
//     planes, or the coupling J_{i+1,i}^T of the next plane on the last one);
//   * a front's vector v_S is h2 on its pivots plus the two halves of its
//     child-contribution slots, which lie in a region of the panel class's
//     own whose entries no child writes stay zero, so no extend-add map is
//     read in the products.
// Nothing a product loads decides a branch: the next chunk's loads stay in
// flight during the current chunk's products.  A workgroup covers 16 RT rows
// (forward) or 16 columns (backward) of one front; its NW waves split the
// contraction into interleaved 16-entry chunks and sum their partial blocks
// through LDS at the end.  Complex products are four real 16 x 16 x 4
// products (FP32 for complex64, FP64 for complex128).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// h2 := the panel's right-hand side in elimination order, 64 positions per
// workgroup and one group of 16 right-hand sides per blockIdx.y.  Mode 0
// writes the panel's own planes (q >= ga); mode 1 writes J_{i+1,i}^T of the
// next plane on the last plane and zeros on the other panel planes.  The
// auxiliary planes (q < ga) are written as zeros: the forward pass adds the
// first children's contributions into this array, so every entry is set
// anew at each solve.
template <typename T>
__global__ __launch_bounds__(256) void k_rhs_scatter(PassArgs<T> A) {
    if (A.run && !*A.run) return;
    __shared__ T Sre[64][17], Sim[64][17];
    const int e0 = blockIdx.x * 64, grp = blockIdx.y;
    const int tid = threadIdx.x, el = tid & 63;
    const int e = e0 + el;
    int64_t goff = -1;
    Cx<double> cf = cx<double>(1, 0);
    if (e < A.naux) {
        const int b = A.perm[e];
        const int q = b / A.NxNy, lat = b - q * A.NxNy;
        if (A.mode == 0) {
            if (q >= A.ga) goff = (int64_t)(A.lo + q - A.ga - A.plane0) * A.NxNy + lat;
        } else if (q == A.nz - 1) {
            goff = (int64_t)(A.hi - A.plane0) * A.NxNy + lat;
            cf = plane_coupling(A, lat);
        }
    }
    // read with consecutive threads on consecutive positions (runs of grid nodes)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = (tid >> 6) + 4 * j;
        const int64_t rr = (int64_t)grp * 16 + r;
        Cx<T> v = cx<T>(0, 0);
        if (goff >= 0 && rr < A.nrhs) {
            const Cx<double> x = A.src[rr * A.ld + goff];
            v = ccast<T>(A.mode == 0 ? x : cf * x);
        }
        Sre[el][r] = v.re;
        Sim[el][r] = v.im;
    }
    __syncthreads();
    // write whole [entry][16] blocks, sixteen consecutive threads per entry
    Cx<T>* h2 = A.h2 + grp * A.gs_h2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int idx = tid + 256 * j;
        const int l = idx >> 4, r = idx & 15;
        if (e0 + l < A.naux) h2[(int64_t)(e0 + l) * 16 + r] = cx<T>(Sre[l][r], Sim[l][r]);
    }
}

// Sum the NW waves' partial 16R x 16 blocks (accumulator layout: lane
// (li, lk) holds column li of rows mfma_out_row(lk, r)) into Y[16R][17].
// When every wave's block fits in the LDS array P (PAR), the waves store
// theirs at once and the workgroup adds them after one barrier; otherwise
// the waves add theirs to Y in turn.  Ends with a barrier.
template <typename T, int R, int NW>
struct WaveSum {
    static constexpr bool PAR = (R == 1 || NW >= 8) && NW * 16 * R * 17 * 2 * (int)sizeof(T) <= 40960;
    static constexpr int PLEN = PAR ? NW * 16 * R * 17 : 1;
};
template <typename T, int R, int NW, typename V4>
__device__ inline void sum_wave_blocks(const V4 (&acr)[R], const V4 (&aci)[R], T (&Yre)[16 * R][17],
                                       T (&Yim)[16 * R][17], T* Pre, T* Pim, int wave, int li, int lk,
                                       int tid) {
    if constexpr (WaveSum<T, R, NW>::PAR) {
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = (wave * 16 * R + 16 * t + mfma_out_row<T>(lk, r)) * 17 + li;
                Pre[o] = acr[t][r];
                Pim[o] = aci[t][r];
            }
        __syncthreads();
        for (int e = tid; e < 16 * R * 16; e += 64 * NW) {
            const int row = e >> 4, c = e & 15;
            T sr = 0, si = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                sr += Pre[(w * 16 * R + row) * 17 + c];
                si += Pim[(w * 16 * R + row) * 17 + c];
            }
            Yre[row][c] = sr;
            Yim[row][c] = si;
        }
        __syncthreads();
    } else {
        for (int w = 0; w < NW; ++w) {
            if (wave == w) {
#pragma unroll
                for (int t = 0; t < R; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * t + mfma_out_row<T>(lk, r);
                        if (w == 0) {
                            Yre[row][li] = acr[t][r];
                            Yim[row][li] = aci[t][r];
                        } else {
                            Yre[row][li] += acr[t][r];
                            Yim[row][li] += aci[t][r];
                        }
                    }
            }
            __syncthreads();
        }
    }
}

// Complex products on the real matrix cores with three real products
// instead of four (the three-multiplication form of the complex product): for
// G = a + ib and v = c + id,
//   k1 += (a + b) c,  k2 += a (d - c),  k3 += b (c + d),
// and then Re(G v) = k1 - k3, Im(G v) = k1 + k2.
template <typename V4>
__device__ inline void cmul3_finish(const V4& k1, const V4& k2, const V4& k3, V4& re, V4& im) {
    re = k1 - k3;
    im = k1 + k2;
}

// An update row's contribution d to the parent (right-hand side r of the
// group): a first child adds it to the parent's right-hand side in h2 where
// it lands on a parent pivot (hm >= 0: the one writer of that entry in the
// launch, so the sum is that of a plain load and store), else it goes to the
// child's half of the parent's slots at position pm.
template <typename T>
__device__ inline void push_update(const PassArgs<T>& A, const SolveItem& it, int grp, int hm, int pm, int r,
                                   Cx<T> d) {
    if (hm >= 0) {
        Cx<T>* h = A.h2 + grp * A.gs_h2 + (int64_t)hm * 16 + r;
        unsafeAtomicAdd(&h->re, d.re);
        unsafeAtomicAdd(&h->im, d.im);
    } else {
        A.c2[grp * A.gs_c2 + (int64_t)(it.push + pm) * 16 + r] = d;
    }
}

// The forward epilogue of one output (row, right-hand side r of the group):
// x_S := D^{-1} y on a pivot row, the update part (the children's
// contributions minus y) to the parent otherwise.
template <typename T>
__device__ inline void fwd_store(const PassArgs<T>& A, const SolveItem& it, int grp, int row, int r, Cx<T> y) {
    const int n = it.n, s = it.s;
    if (row >= n) return;
    if (row < s) {
        if (row >= leaf_aux_rows(it, A.ga))
            A.xu[grp * A.gs_u + (int64_t)(it.xu - s + row) * 16 + r] = y * A.dinv[it.start + row];
    } else {
        const Cx<T>* c2f = A.c2 + grp * A.gs_c2 + (int64_t)it.c2 * 16;
        const Cx<T> pre = it.leaf ? cx<T>(0, 0) : c2f[(int64_t)row * 16 + r] + c2f[(int64_t)(n + row) * 16 + r];
        push_update(A, it, grp, A.hmap[it.pmap + row - s], A.pmap[it.pmap + row - s], r, pre - y);
    }
}

// RT row tiles of 16 per workgroup: each of the NW waves updates all of them
// over every NW-th chunk of the contraction.  Launches with few workgroups
// (the upper depths, with long contractions) take the wide form, NW = 8, to
// shorten each wave's chain of chunks.
// SK: split contraction.  Workgroup b takes item b / nsplit and the
// (b mod nsplit)-th share of its chunks and stores its partial block; a
// finishing launch (k_fwd_fin) sums the shares.
template <typename T, int RT, int NW, int SK = 0>
__global__ __launch_bounds__(64 * NW) void k_fwd_mm(PassArgs<T> A) {
    typedef typename MfmaAcc<T>::type V4;
    constexpr int KC = 16;
    static_assert(SK == 0 || NW == 4, "split contraction: 4 waves (one thread per partial entry)");
    const int S = SK != 0 ? A.nsplit : 1;
    const int ib = SK != 0 ? (int)blockIdx.x / S : (int)blockIdx.x;
    const int z = SK != 0 ? (int)blockIdx.x - ib * S : 0;
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[ib];  // items of 16 RT rows
    if (it.blk + 16 * RT <= leaf_aux_rows(it, A.ga)) return;  // nothing to store
    const int n = it.n, s = it.s;
    const int grp = blockIdx.y;
    const int64_t rhs0 = (int64_t)grp * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int kend = (it.blk + 16 * RT <= s) ? it.blk + 16 * RT : s;
    __shared__ T Yre[16 * RT][17], Yim[16 * RT][17];  // the block's sum [row][rhs]
    // the front's slices of the group: children's halves [0, n) and [n, 2n),
    // right-hand side on its pivots
    const Cx<T>* c2f = A.c2 + grp * A.gs_c2 + (int64_t)it.c2 * 16;
    const Cx<T>* h2f = A.h2 + grp * A.gs_h2 + (int64_t)it.start * 16;
    constexpr uint32_t ES = sizeof(Cx<T>);
    // Operand descriptors cut at the contraction's end kend: G's first kend
    // columns and the first kend entries of each part of v_S.  Loads past
    // them read zeros, so every chunk issues the same loads (the next
    // chunk's stay in flight during this one's products) and needs no bounds
    // test; rows past n give product rows that are never stored.
    // v_S is h2 (the right-hand side, to which the first child has added its
    // contributions on these pivots) plus the second child's half; a leaf has
    // h2 alone.
    const uint32_t c2len = it.leaf ? 0u : (uint32_t)kend * 16 * ES;
    const BufRsrc rg = buf_rsrc(A.G + it.loff, (uint32_t)kend * n * ES);
    const BufRsrc rh = buf_rsrc(h2f, (uint32_t)kend * 16 * ES);
    const BufRsrc r1 = buf_rsrc(c2f + (int64_t)n * 16, c2len);
    // With one row tile, the epilogue's operands (1/D of a pivot row, or the
    // children's contributions and the parent position of an update row)
    // are loaded first, bounded so that every load is unconditional: they
    // arrive during the products instead of after them.
    const int erow = it.blk + (tid >> 4), er = tid & 15;
    Cx<T> e_d = cx<T>(0, 0), e_a = cx<T>(0, 0), e_b = cx<T>(0, 0);
    int e_pm = 0, e_hm = -1;
    if constexpr (RT == 1 && NW >= 4) {
        const BufRsrc rd = buf_rsrc(A.dinv + it.start, (uint32_t)s * ES);
        const BufRsrc rp = buf_rsrc(A.pmap + it.pmap, (uint32_t)(n - s) * 4);
        const BufRsrc rm = buf_rsrc(A.hmap + it.pmap, (uint32_t)(n - s) * 4);
        const BufRsrc rc = buf_rsrc(c2f, it.leaf ? 0u : (uint32_t)(2 * n) * 16 * ES);
        BufCx<T>::load(rd, (uint32_t)erow * ES, e_d.re, e_d.im);
        e_pm = buf_load_i32(rp, (uint32_t)(erow - s) * 4);
        e_hm = buf_load_i32(rm, (uint32_t)(erow - s) * 4);
        BufCx<T>::load(rc, (uint32_t)(erow * 16 + er) * ES, e_a.re, e_a.im);
        BufCx<T>::load(rc, (uint32_t)((n + erow) * 16 + er) * ES, e_b.re, e_b.im);
    }
    // lane operands: A(row, k) = G(blk + 16 t + li, c + 4 q + lk) and
    // B(k, rhs) = v_S(c + 4 q + lk, li)
    T gre[RT][4], gim[RT][4];
    T vre[2][4], vim[2][4];
    // np: the parts of v_S loaded (a leaf has the right-hand side alone, and
    // its loop issues no loads of the empty child slots)
    auto load = [&](auto np, int c, T(&gr)[RT][4], T(&gi)[RT][4], T(&br)[2][4], T(&bi)[2][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t col = (uint32_t)(c + 4 * q + lk);
#pragma unroll
            for (int t = 0; t < RT; ++t)
                BufCx<T>::load(rg, (col * n + it.blk + 16 * t + li) * ES, gr[t][q], gi[t][q]);
            const uint32_t vo = (col * 16 + li) * ES;
            BufCx<T>::load(rh, vo, br[0][q], bi[0][q]);
            if constexpr (decltype(np)::value == 2)
                BufCx<T>::load(r1, vo, br[1][q], bi[1][q]);
            else
                br[1][q] = bi[1][q] = 0;
        }
    };
    // complex products with three real ones (cmul3): three independent
    // accumulator chains per row tile
    V4 k1[RT], k2[RT], k3[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) k1[t] = k2[t] = k3[t] = V4{0, 0, 0, 0};
    // chunks from the one holding the first live pivot (entries before it are zeros)
    const int kb = (leaf_first_live(A, it) / KC) * KC;
    const int nch = kend > kb ? (kend - kb + KC - 1) / KC : 0;
    auto products = [&](const T(&gr)[RT][4], const T(&gi)[RT][4], const T(&vr)[2][4], const T(&vi)[2][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T br = vr[0][q] + vr[1][q], bi = vi[0][q] + vi[1][q];
            const T bs = br + bi, bd = bi - br;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                k1[t] = mfma4(gr[t][q] + gi[t][q], br, k1[t]);
                k2[t] = mfma4(gr[t][q], bd, k2[t]);
                k3[t] = mfma4(gi[t][q], bs, k3[t]);
            }
        }
    };
    // one chunk at a time per wave: the loads of the waves sharing a SIMD
    // overlap each other's products (a few waves per SIMD at this register
    // count); a load past the contraction's end reads zeros.  (Two chunks in
    // flight per wave, their loads kept ahead of the products, measured
    // slower at every depth.)
    const int per = (nch + S - 1) / S, c_lo = z * per, c_hi = min(nch, c_lo + per);
    auto chunks = [&](auto np) {
        for (int ch = c_lo + wave; ch < c_hi; ch += NW) {
            load(np, kb + ch * KC, gre, gim, vre, vim);
            products(gre, gim, vre, vim);
        }
    };
    if (it.leaf)
        chunks(std::integral_constant<int, 1>{});
    else
        chunks(std::integral_constant<int, 2>{});
    // sum the waves' partial blocks
    {
        __shared__ T Pre[WaveSum<T, RT, NW>::PLEN], Pim[WaveSum<T, RT, NW>::PLEN];
        V4 acr[RT], aci[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) cmul3_finish(k1[t], k2[t], k3[t], acr[t], aci[t]);
        sum_wave_blocks<T, RT, NW>(acr, aci, Yre, Yim, Pre, Pim, wave, li, lk, tid);
    }
    if constexpr (SK != 0) {
        Cx<T>* pp = A.part + ((int64_t)(ib * gridDim.y + grp) * S + z) * (256 * RT);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int e = tid + 256 * t;
            pp[e] = cx<T>(Yre[e >> 4][e & 15], Yim[e >> 4][e & 15]);
        }
        return;
    }
    if constexpr (NW < 4) {
        // fewer than 256 threads: each takes several (row, right-hand side) outputs
        for (int idx = tid; idx < 256 * RT; idx += 64 * NW) {
            const int rr = idx & 15;
            if (rhs0 + rr < A.nrhs)
                fwd_store(A, it, grp, it.blk + (idx >> 4), rr, cx<T>(Yre[idx >> 4][rr], Yim[idx >> 4][rr]));
        }
        return;
    }
    // thread tid < 256: right-hand side rhs0 + tid % 16 of rows blk + tid / 16 + 16 t
    // (a row's 16 right-hand sides are one contiguous block)
    const int r = tid & 15;
    if (tid >= 256 || rhs0 + r >= A.nrhs) return;
    Cx<T>* xs = A.xu + grp * A.gs_u + (int64_t)(it.xu - s) * 16;  // the front's [x_S; -x_U]
    Cx<T>* c2g = A.c2 + grp * A.gs_c2;
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int lrow = (tid >> 4) + 16 * t, row = it.blk + lrow;
        if (row >= n) continue;
        const Cx<T> y = cx<T>(Yre[lrow][r], Yim[lrow][r]);
        if constexpr (RT == 1) {
            if (row < s) {
                if (row >= leaf_aux_rows(it, A.ga)) xs[(int64_t)row * 16 + r] = y * e_d;
            } else {
                push_update(A, it, grp, e_hm, e_pm, r, (e_a + e_b) - y);
            }
        } else {
            fwd_store(A, it, grp, row, r, y);
        }
    }
}

// y[t] := sum over the S partial blocks at pp (256 R entries apart) of entry
// tid + 256 t, added in split order; the loads of eight splits are issued
// before their sums.
template <typename T, int R>
__device__ inline void split_sums(const Cx<T>* pp, int S, int tid, Cx<T> (&y)[R]) {
#pragma unroll
    for (int t = 0; t < R; ++t) y[t] = cx<T>(0, 0);
    for (int z0 = 0; z0 < S; z0 += 8) {
        Cx<T> v[8][R];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int t = 0; t < R; ++t)  // unconditional loads (clamped split, dropped below)
                v[u][t] = pp[(int64_t)min(z0 + u, S - 1) * (256 * R) + tid + 256 * t];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int t = 0; t < R; ++t)
                if (z0 + u < S) y[t] = y[t] + v[u][t];
    }
}

// Sums the nsplit partial blocks of each item of 16 RT rows (in split order,
// so the result does not depend on timing) and applies the forward epilogue.
template <typename T, int RT>
__global__ __launch_bounds__(256) void k_fwd_fin(PassArgs<T> A) {
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    const int grp = blockIdx.y, tid = threadIdx.x, r = tid & 15, S = A.nsplit;
    if ((int64_t)grp * 16 + r >= A.nrhs) return;
    Cx<T> y[RT];
    split_sums<T, RT>(A.part + (int64_t)(blockIdx.x * gridDim.y + grp) * S * (256 * RT), S, tid, y);
#pragma unroll
    for (int t = 0; t < RT; ++t) fwd_store(A, it, grp, it.blk + ((tid + 256 * t) >> 4), r, y[t]);
}

// Row-split form of the forward matrix-core pass for fronts whose v_S fits
// in LDS: the workgroup's 64 rows go one 16-row tile to each of its four
// waves, so no partial sums are combined.  The workgroup stages its slice of
// v_S (right-hand side, which holds the first child's part, plus the second
// child's half, summed) once in LDS, together with what the epilogue needs
// (1/D of its pivot rows, the children's contributions and parent positions
// of its update rows); each
// wave then streams its rows of G with FP chunks of loads in flight, taking
// the B operand from LDS.  The first FP chunks are issued before the staging
// loads.  LDS: fwd_rs_lds_bytes.
template <typename T, int FP>
__global__ __launch_bounds__(256) void k_fwd_rs(PassArgs<T> A) {
    typedef typename MfmaAcc<T>::type V4;
    constexpr int KC = 16, ROWS = 64;
    constexpr uint32_t ES = sizeof(Cx<T>);
    extern __shared__ unsigned char smem_raw[];
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];  // items of 64 rows
    if (it.blk + ROWS <= leaf_aux_rows(it, A.ga)) return;  // nothing to store
    const int n = it.n, s = it.s;
    const int grp = blockIdx.y;
    const int64_t rhs0 = (int64_t)grp * 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: G's descriptor is scalar
    const int li = lane & 15, lk = lane >> 4;
    const int kend = min(it.blk + ROWS, s);
    const int kb = (leaf_first_live(A, it) / KC) * KC;
    const int nk16 = kend > kb ? (kend - kb + KC - 1) / KC * KC : 0;  // staged entries
    Cx<T>* V = reinterpret_cast<Cx<T>*>(smem_raw);   // [nk16][16]
    Cx<T>* E = V + (int64_t)nk16 * 16;               // [ROWS][16]
    Cx<T>* Dv = E + ROWS * 16;                       // [ROWS]
    int* PM = reinterpret_cast<int*>(Dv + ROWS);     // [ROWS]
    int* HM = PM + ROWS;                             // [ROWS], then one spare entry
    const Cx<T>* c2f = A.c2 + grp * A.gs_c2 + (int64_t)it.c2 * 16;
    const Cx<T>* h2f = A.h2 + grp * A.gs_h2 + (int64_t)it.start * 16;
    // this wave's rows r0 .. r0 + 15 need the columns below kw (the triangle
    // of L_F^{-1} above; all s columns for update rows); its G descriptor is
    // cut there, so the chunks issued past its end read zeros without
    // touching memory
    const int r0 = it.blk + 16 * wave;
    const int kw = r0 < n ? min(r0 + 16, s) : 0;
    const int nch = kw > kb ? (kw - kb + KC - 1) / KC : 0;
    const BufRsrc rg = buf_rsrc(A.G + it.loff, (uint32_t)kw * n * ES);
    T gre[FP][4], gim[FP][4];
    auto load = [&](int ch, T(&gr)[4], T(&gi)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t col = (uint32_t)(kb + ch * KC + 4 * q + lk);
            BufCx<T>::load(rg, (col * n + r0 + li) * ES, gr[q], gi[q]);
        }
    };
#pragma unroll
    for (int j = 0; j < FP; ++j) load(j, gre[j], gim[j]);
    // Staging.  Every load is unconditional and bounded by its descriptor
    // (reads past the end give zeros), and values no one needs are stored to
    // a spare LDS slot, so no load waits on a branch: the epilogue operands
    // of the workgroup's rows, then v_S over [kb, kb + nk16) (zeros from kend
    // on), summed from the right-hand side and the children's halves.
    {
        const uint32_t c2len = it.leaf ? 0u : (uint32_t)kend * 16 * ES;
        const uint32_t c2all = it.leaf ? 0u : (uint32_t)n * 16 * ES;
        const BufRsrc rh = buf_rsrc(h2f, (uint32_t)kend * 16 * ES);
        const BufRsrc rb = buf_rsrc(c2f + (int64_t)n * 16, c2len);
        const BufRsrc ea = buf_rsrc(c2f, c2all), eb = buf_rsrc(c2f + (int64_t)n * 16, c2all);
        const BufRsrc rd = buf_rsrc(A.dinv + it.start, (uint32_t)s * ES);
        const BufRsrc rp = buf_rsrc(A.pmap + it.pmap, (uint32_t)(n - s) * 4);
        const BufRsrc rm = buf_rsrc(A.hmap + it.pmap, (uint32_t)(n - s) * 4);
        T er[4], ei[4], fr[4], fi[4], dr, di;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u, row = it.blk + (e >> 4);
            const uint32_t off = (uint32_t)(row * 16 + (e & 15)) * ES;
            BufCx<T>::load(ea, off, er[u], ei[u]);
            BufCx<T>::load(eb, off, fr[u], fi[u]);
        }
        const int drow = it.blk + (tid & 63);
        BufCx<T>::load(rd, (uint32_t)drow * ES, dr, di);  // zero from s on
        const int pm = buf_load_i32(rp, (uint32_t)(drow - s) * 4);  // zero on pivot rows
        const int hm = buf_load_i32(rm, (uint32_t)(drow - s) * 4);
        Cx<T>* trash = reinterpret_cast<Cx<T>*>(HM + ROWS);  // 512 bytes past PM: aligned
        const int tot = nk16 * 16;
        constexpr int SU = 4;  // entries per thread and round
        auto stage = [&](auto np) {  // np: parts of v_S (a leaf: the right-hand side alone)
            for (int e0 = tid; e0 < tot; e0 += SU * 256) {
                T hr[SU], hi[SU], br[SU], bi[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const uint32_t off = (uint32_t)(kb * 16 + e0 + 256 * u) * ES;
                    BufCx<T>::load(rh, off, hr[u], hi[u]);
                    if constexpr (decltype(np)::value == 2)
                        BufCx<T>::load(rb, off, br[u], bi[u]);
                    else
                        br[u] = bi[u] = 0;
                }
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int e = e0 + 256 * u;
                    *(e < tot ? V + e : trash) = cx<T>(hr[u] + br[u], hi[u] + bi[u]);
                }
            }
        };
        if (it.leaf)
            stage(std::integral_constant<int, 1>{});
        else
            stage(std::integral_constant<int, 2>{});
        // pivot rows take no contribution (their slots hold the children's
        // v_S parts, already summed above)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u, row = it.blk + (e >> 4);
            E[e] = row >= s ? cx<T>(er[u] + fr[u], ei[u] + fi[u]) : cx<T>(0, 0);
        }
        if (tid < ROWS) {
            Dv[tid] = cx<T>(dr, di);
            PM[tid] = pm;
            HM[tid] = hm;
        }
    }
    __syncthreads();
    V4 k1 = V4{0, 0, 0, 0}, k2 = V4{0, 0, 0, 0}, k3 = V4{0, 0, 0, 0};  // cmul3
    auto products = [&](int ch, const T(&gr)[4], const T(&gi)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const Cx<T> v = V[(ch * KC + 4 * q + lk) * 16 + li];
            k1 = mfma4(gr[q] + gi[q], v.re, k1);
            k2 = mfma4(gr[q], v.im - v.re, k2);
            k3 = mfma4(gi[q], v.re + v.im, k3);
        }
    };
    // chunk ch + j sits in buffer j; each buffer is refilled with the chunk
    // FP ahead as soon as its products are issued
    for (int ch = 0; ch < nch; ch += FP) {
#pragma unroll
        for (int j = 0; j < FP; ++j) {
            if (ch + j < nch) products(ch + j, gre[j], gim[j]);
            load(ch + j + FP, gre[j], gim[j]);
        }
    }
    V4 a0, b0;
    cmul3_finish(k1, k2, k3, a0, b0);
    if (rhs0 + li >= A.nrhs) return;
    Cx<T>* xs = A.xu + grp * A.gs_u + (int64_t)(it.xu - s) * 16;  // the front's [x_S; -x_U]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lrow = 16 * wave + mfma_out_row<T>(lk, r), row = it.blk + lrow;
        if (row >= n) continue;
        const Cx<T> y = cx<T>(a0[r], b0[r]);
        if (row < s) {
            if (row >= leaf_aux_rows(it, A.ga)) xs[(int64_t)row * 16 + li] = y * Dv[lrow];
        } else {
            push_update(A, it, grp, HM[lrow], PM[lrow], li, E[lrow * 16 + li] - y);
        }
    }
}

// LDS of k_fwd_rs for fronts of up to smax pivots (staged v_S, the
// epilogue's contributions, 1/D and the two parent position maps).
template <typename T>
size_t fwd_rs_lds_bytes(int smax) {
    const size_t nk16 = (size_t)(smax + 15) / 16 * 16;
    return (nk16 * 16 + 64 * 16 + 64 + 1) * sizeof(Cx<T>) + 2 * 64 * sizeof(int);
}

// CT column tiles of 16 per workgroup; NW waves split the rows of the
// contraction by chunks (the wide form, CT = 1 and more waves, serves
// launches with few workgroups).  The contraction index of each 16-row chunk
// is relabelled so that lane (li, lk) of the four products m = 0..3 holds
// rows i0 + 4 lk + m: a lane then reads four consecutive rows of one column
// of G in one access, and sixteen lanes read one 128-byte run of [x_S; -x_U],
// so both operands come straight from memory, with no LDS staging.
// The backward epilogue: x_S(j) of right-hand side r of the group goes to
// the children's update-set values (stored negated: a front's vector holds
// [x_S; -x_U]) ...
template <typename T>
__device__ inline void bwd_push(const PassArgs<T>& A, const SolveItem& it, int grp, int j, int r, Cx<T> x) {
    Cx<T>* xu = A.xu + grp * A.gs_u;
    if (it.cxu0 >= 0) {
        const int o0 = A.cmap[it.moff + j];
        if (o0 >= 0) xu[(int64_t)(it.cxu0 + o0) * 16 + r] = -x;
    }
    if (it.cxu1 >= 0) {
        const int o1 = A.cmap[it.moff + it.n + j];
        if (o1 >= 0) xu[(int64_t)(it.cxu1 + o1) * 16 + r] = -x;
    }
}
// ... and (right-hand side orr) to the panel's planes of the padded grid:
// stored (mode 0, with the coupling into the next plane when asked) or
// subtracted (mode 1).
template <typename T>
__device__ inline void bwd_grid(const PassArgs<T>& A, const SolveItem& it, int j, int64_t orr, Cx<T> x) {
    const int b = pivot_box(it, A.Nx, A.NxNy, j);
    const int q = b / A.NxNy, lat = b - q * A.NxNy;
    if (q < A.ga) return;
    Cx<double>* up = A.dst + orr * A.ld + (int64_t)(A.lo + q - A.ga - A.plane0) * A.NxNy + lat;
    const Cx<double> xd = ccast<double>(x);
    if (A.mode == 0) {
        *up = xd;
        if (A.couple && q == A.nz - 1) up[A.NxNy] = up[A.NxNy] - plane_coupling(A, lat) * xd;
    } else {
        *up = *up - xd;
    }
}

// SK: split contraction.  Workgroup b takes item b / nsplit and the
// (b mod nsplit)-th share of its row chunks (and of the front's hand-on)
// and stores its partial block; a finishing launch (k_bwd_fin) sums the
// shares.
// IFB: chunks in flight per wave with one column tile (their loads all
// issued before their products).
template <typename T, int CT, int NW, int SK = 0, int IFB = 2>
__global__ __launch_bounds__(64 * NW) void k_bwd_mm(PassArgs<T> A) {
    typedef typename MfmaAcc<T>::type V4;
    constexpr int KC = 16;
    static_assert(SK == 0 || NW == 4, "split contraction: 4 waves (one thread per partial entry)");
    static_assert(IFB == 2 || (IFB == 4 && CT == 1), "four chunks in flight: one column tile");
    const int S = SK != 0 ? A.nsplit : 1;
    const int ib = SK != 0 ? (int)blockIdx.x / S : (int)blockIdx.x;
    const int z = SK != 0 ? (int)blockIdx.x - ib * S : 0;
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[ib];  // items of 16 CT columns
    if (leaf_aux_block(it, A.ga, it.blk, 16 * CT)) return;
    const int n = it.n, s = it.s;
    const int grp = blockIdx.y;
    const int64_t rhs0 = (int64_t)grp * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int c0 = it.blk;
    __shared__ T Yre[16 * CT][17], Yim[16 * CT][17];  // the waves' partial blocks, summed [column][rhs]
    // the front's [x_S; -x_U]: x_S from the forward pass, -x_U from the
    // parent's backward pass (entry i at xsu + 16 i, the x_U part at xuf)
    Cx<T>* xu = A.xu + grp * A.gs_u;
    const Cx<T>* xsu = xu + (int64_t)(it.xu - s) * 16;
    const Cx<T>* xuf = xu + (int64_t)it.xu * 16;
    // With one column tile, the epilogue's operands that do not depend on the
    // products -- the children's positions of the block's pivots and the
    // padded grid's old value (subtracted from in mode 1, the next plane's
    // in mode 0 with the coupling) -- are loaded first and unconditionally
    // (bounded descriptor, or the grid's base address where nothing is read
    // back), so they arrive during the products.
    int e_o0 = -1, e_o1 = -1;
    Cx<double> e_old = cx<double>(0, 0);
    Cx<double>* e_up = nullptr;
    int e_q = -1, e_lat = 0;
    if constexpr (CT == 1 && NW >= 4) {
        const BufRsrc rm = buf_rsrc(A.cmap + it.moff, (uint32_t)(2 * n) * 4);
        const int jc = c0 + (tid >> 4) % 16;
        e_o0 = buf_load_i32(rm, (uint32_t)jc * 4);
        e_o1 = buf_load_i32(rm, (uint32_t)(n + jc) * 4);
        const int j = c0 + (tid & 15);
        const int64_t orr = rhs0 + ((tid >> 4) & 15);
        const int b = pivot_box(it, A.Nx, A.NxNy, j);
        e_q = b / A.NxNy;
        e_lat = b - e_q * A.NxNy;
        const bool ok = j < s && orr < A.nrhs && e_q >= A.ga;
        e_up = A.dst + orr * A.ld + (int64_t)(A.lo + e_q - A.ga - A.plane0) * A.NxNy + e_lat;
        const bool rd = ok && (A.mode != 0 || (A.couple && e_q == A.nz - 1));
        const Cx<double>* src = rd ? (A.mode != 0 ? e_up : e_up + A.NxNy) : A.dst;
        e_old = *src;
    }
    // The update-set values go on to the children.  The front's column blocks
    // share its u rows, sixteen threads per row (one per right-hand side),
    // and each thread issues the loads of four rows before their stores, so
    // the map lookups do not form one long chain of memory round trips.
    if (it.cxu0 >= 0 || it.cxu1 >= 0) {
        const int u = n - s;
        const int nb = (s + 16 * CT - 1) / (16 * CT) * S, b = c0 / (16 * CT) * S + z;
        const int per = (u + nb - 1) / nb;
        const int i_lo = s + b * per, i_hi = min(n, i_lo + per);
        constexpr int ROWS = 4 * NW;  // rows per pass of the workgroup
        const int r = tid & 15;
        for (int i0 = i_lo + (tid >> 4); i0 < i_hi; i0 += 4 * ROWS) {
            Cx<T> xv[4];
            int p0[4], p1[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * ROWS;
                const bool ok = i < i_hi;
                p0[k] = ok && it.cxu0 >= 0 ? A.cmap[it.moff + i] : -1;
                p1[k] = ok && it.cxu1 >= 0 ? A.cmap[it.moff + n + i] : -1;
                xv[k] = ok ? xuf[(int64_t)(i - s) * 16 + r] : cx<T>(0, 0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (p0[k] >= 0) xu[(int64_t)(it.cxu0 + p0[k]) * 16 + r] = xv[k];
                if (p1[k] >= 0) xu[(int64_t)(it.cxu1 + p1[k]) * 16 + r] = xv[k];
            }
        }
    }
    // Operand descriptors cut at the front's ends: G's s columns and the n
    // entries of [x_S; -x_U].  Loads past them read zeros, so no chunk tests
    // bounds; columns past s give results never stored.
    constexpr uint32_t ES = sizeof(Cx<T>);
    const BufRsrc rg = buf_rsrc(A.G + it.loff, (uint32_t)s * n * ES);
    const BufRsrc rs = buf_rsrc(xsu, (uint32_t)n * 16 * ES);
    T gre[CT][4], gim[CT][4], sre[4], sim[4];
    V4 k1[CT], k2[CT], k3[CT];  // cmul3, as in k_fwd_mm
#pragma unroll
    for (int t = 0; t < CT; ++t) k1[t] = k2[t] = k3[t] = V4{0, 0, 0, 0};
    // rows above the block's first column are zeros of G_TL; a leaf's
    // auxiliary rows are skipped (leaf_aux_rows)
    const int ib0 = max(c0, leaf_aux_rows(it, A.ga));
    const int nch = (n - ib0 + KC - 1) / KC;
    // this lane's four rows i0 .. i0 + 3 of chunk ch
    auto load = [&](int ch, T(&gr)[CT][4], T(&gi)[CT][4], T(&sr)[4], T(&si)[4]) {
        const int i0 = ib0 + ch * KC + 4 * lk;
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const uint32_t off = ((uint32_t)(c0 + 16 * t + li) * n + (uint32_t)i0) * ES;
#pragma unroll
            for (int m = 0; m < 4; ++m) BufCx<T>::load(rg, off + m * ES, gr[t][m], gi[t][m]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) BufCx<T>::load(rs, (uint32_t)((i0 + m) * 16 + li) * ES, sr[m], si[m]);
    };
    auto products = [&](const T(&gr)[CT][4], const T(&gi)[CT][4], const T(&sr)[4], const T(&si)[4]) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const T br = sr[m], bi = si[m];
            const T bs = br + bi, bd = bi - br;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                k1[t] = mfma4(gr[t][m] + gi[t][m], br, k1[t]);
                k2[t] = mfma4(gr[t][m], bd, k2[t]);
                k3[t] = mfma4(gi[t][m], bs, k3[t]);
            }
        }
    };
    // with one column tile each wave issues two chunks' loads before their
    // products (loads past the end read zeros), as in k_fwd_mm
    if constexpr (SK == 0 && CT == 1 && IFB == 4) {
        T gre2[CT][4], gim2[CT][4], sre2[4], sim2[4], gre3[CT][4], gim3[CT][4], sre3[4], sim3[4];
        T gre4[CT][4], gim4[CT][4], sre4[4], sim4[4];
        for (int ch = wave; ch < nch; ch += 4 * NW) {
            load(ch, gre, gim, sre, sim);
            load(ch + NW, gre2, gim2, sre2, sim2);
            load(ch + 2 * NW, gre3, gim3, sre3, sim3);
            load(ch + 3 * NW, gre4, gim4, sre4, sim4);
            __builtin_amdgcn_sched_barrier(0);  // all four chunks' loads ahead of the products
            products(gre, gim, sre, sim);
            products(gre2, gim2, sre2, sim2);
            products(gre3, gim3, sre3, sim3);
            products(gre4, gim4, sre4, sim4);
        }
    } else if constexpr (SK == 0 && CT == 1) {
        T gre2[CT][4], gim2[CT][4], sre2[4], sim2[4];
        for (int ch = wave; ch < nch; ch += 2 * NW) {
            load(ch, gre, gim, sre, sim);
            load(ch + NW, gre2, gim2, sre2, sim2);
            __builtin_amdgcn_sched_barrier(0);  // both chunks' loads ahead of the products
            products(gre, gim, sre, sim);
            products(gre2, gim2, sre2, sim2);
        }
    } else {
        const int per = (nch + S - 1) / S, c_lo = z * per, c_hi = min(nch, c_lo + per);
        for (int ch = c_lo + wave; ch < c_hi; ch += NW) {
            load(ch, gre, gim, sre, sim);
            products(gre, gim, sre, sim);
        }
    }
    // sum the waves' partial blocks
    {
        __shared__ T Pre[WaveSum<T, CT, NW>::PLEN], Pim[WaveSum<T, CT, NW>::PLEN];
        V4 acr[CT], aci[CT];
#pragma unroll
        for (int t = 0; t < CT; ++t) cmul3_finish(k1[t], k2[t], k3[t], acr[t], aci[t]);
        sum_wave_blocks<T, CT, NW>(acr, aci, Yre, Yim, Pre, Pim, wave, li, lk, tid);
    }
    if constexpr (SK != 0) {
        Cx<T>* pp = A.part + ((int64_t)(ib * gridDim.y + grp) * S + z) * (256 * CT);
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int e = tid + 256 * t;
            pp[e] = cx<T>(Yre[e >> 4][e & 15], Yim[e >> 4][e & 15]);
        }
        return;
    }
    if constexpr (NW < 4) {
        // fewer than 256 threads: each takes several (column, right-hand side) outputs
        for (int idx = tid; idx < 256 * CT; idx += 64 * NW) {
            const int jl = idx >> 4, rr = idx & 15, j = c0 + jl;
            if (j < s && rhs0 + rr < A.nrhs) {
                const Cx<T> x = cx<T>(Yre[jl][rr], Yim[jl][rr]);
                bwd_push(A, it, grp, j, rr, x);
                bwd_grid(A, it, j, rhs0 + rr, x);
            }
        }
        return;
    }
    if (tid >= 256) return;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        // children's update-set values: a column's 16 right-hand sides are one block
        {
            const int jl = 16 * t + (tid >> 4), r = tid & 15, j = c0 + jl;
            if (j < s && rhs0 + r < A.nrhs) {
                const Cx<T> x = cx<T>(Yre[jl][r], Yim[jl][r]);
                if constexpr (CT == 1) {
                    if (it.cxu0 >= 0 && e_o0 >= 0) xu[(int64_t)(it.cxu0 + e_o0) * 16 + r] = -x;
                    if (it.cxu1 >= 0 && e_o1 >= 0) xu[(int64_t)(it.cxu1 + e_o1) * 16 + r] = -x;
                } else {
                    bwd_push(A, it, grp, j, r, x);
                }
            }
        }
        // the padded grid: consecutive threads on consecutive pivots of one right-hand side
        const int jl = 16 * t + (tid & 15), j = c0 + jl;
        const int64_t orr = rhs0 + (tid >> 4);
        if (j >= s || orr >= A.nrhs) continue;
        const Cx<T> x = cx<T>(Yre[jl][tid >> 4], Yim[jl][tid >> 4]);
        const Cx<double> xd = ccast<double>(x);
        if constexpr (CT == 1) {
            if (e_q < A.ga) continue;
            if (A.mode == 0) {
                *e_up = xd;
                if (A.couple && e_q == A.nz - 1) e_up[A.NxNy] = e_old - plane_coupling(A, e_lat) * xd;
            } else {
                *e_up = e_old - xd;
            }
        } else {
            bwd_grid(A, it, j, orr, x);
        }
    }
}

// Sums the nsplit partial blocks of each item of 16 CT columns (in split
// order) and applies the backward epilogue.
template <typename T, int CT>
__global__ __launch_bounds__(256) void k_bwd_fin(PassArgs<T> A) {
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    if (leaf_aux_block(it, A.ga, it.blk, 16 * CT)) return;
    const int grp = blockIdx.y, tid = threadIdx.x, S = A.nsplit;
    const int64_t rhs0 = (int64_t)grp * 16;
    __shared__ T Yre[16 * CT][17], Yim[16 * CT][17];
    Cx<T> y[CT];
    split_sums<T, CT>(A.part + (int64_t)(blockIdx.x * gridDim.y + grp) * S * (256 * CT), S, tid, y);
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int e = tid + 256 * t;
        Yre[e >> 4][e & 15] = y[t].re;
        Yim[e >> 4][e & 15] = y[t].im;
    }
    __syncthreads();
    const int s = it.s, c0 = it.blk;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        {
            const int jl = 16 * t + (tid >> 4), r = tid & 15, j = c0 + jl;
            if (j < s && rhs0 + r < A.nrhs) bwd_push(A, it, grp, j, r, cx<T>(Yre[jl][r], Yim[jl][r]));
        }
        const int jl = 16 * t + (tid & 15), j = c0 + jl;
        const int64_t orr = rhs0 + (tid >> 4);
        if (j < s && orr < A.nrhs) bwd_grid(A, it, j, orr, cx<T>(Yre[jl][tid >> 4], Yim[jl][tid >> 4]));
    }
}

// ---------------------------------------------------------------------------
// Triangular passes with the factors themselves, the path selective
// inversion replaces (Sec. 2.2): the forward step x_S := L_F^{-1} x_S,
// x_U := x_U - F_BL x_S and the backward step x_S := L_F^{-T}(x_S - F_BL^T
// x_U), by 64-pivot blocks in order.  L = [L_F; F_BL] is the kept factor
// block (n x s, column-major, the layout of G); each 64 x 64 diagonal block of
// L_F holds above its diagonal the inverse X of its unit lower part, X(r, c)
// (r > c) at row c, column r of the block, as the factorisation left it.
// One workgroup of TRI_NT threads per (front, right-hand-side chunk); inputs,
// outputs and the exchanges between fronts are those of k_fwd / k_bwd.
constexpr int TRI_NT = 256;

template <typename T, int RC>
__global__ __launch_bounds__(TRI_NT) void k_fwd_tri(PassArgs<T> A) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* v = reinterpret_cast<Cx<T>*>(smem_raw);  // [RC][n]: the front vector, then x
    __shared__ Cx<T> xb[RC][64];
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    const int n = it.n, s = it.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, A.nrhs - rhs0);
    const int tid = threadIdx.x;
    const Cx<T>* L = A.G + it.loff;
    const int* map0 = A.cmap + it.moff;
    const int* map1 = map0 + n;
    // children's contributions on every row of the front, plus the
    // right-hand side on its pivots (slots a child does not cover are masked)
    for (int k = tid; k < n; k += TRI_NT) {
        const bool h0 = map0[k] >= 0, h1 = map1[k] >= 0;
        bool live = false;
        int64_t gi = 0;
        Cx<double> cf = cx<double>(1, 0);
        if (k < s) {
            const int b = pivot_box(it, A.Nx, A.NxNy, k);
            const int q = b / A.NxNy, lat = b - q * A.NxNy;
            if (A.mode == 0) {
                live = q >= A.ga;
                gi = (int64_t)(A.lo + q - A.ga - A.plane0) * A.NxNy + lat;
            } else {
                live = q == A.nz - 1;
                gi = (int64_t)(A.hi - A.plane0) * A.NxNy + lat;
                if (live) cf = plane_coupling(A, lat);
            }
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            Cx<T> val = cx<T>(0, 0);
            if (r < nr) {
                const int64_t rr = rhs0 + r;
                const Cx<T>* cc = A.c2 + rr * A.c2ld + it.c2;
                val = keep(h0, cc[k]) + keep(h1, cc[n + k]);
                if (live) {
                    const Cx<double> x = A.src[rr * A.ld + gi];
                    val = val + ccast<T>(A.mode == 0 ? x : cf * x);
                }
            }
            v[r * n + k] = val;
        }
    }
    __syncthreads();
    // a leaf's vector is zero before its first live pivot: those blocks stay zero
    for (int b0 = leaf_first_live(A, it) / 64 * 64; b0 < s; b0 += 64) {
        const int bw = min(64, s - b0);
        {   // x_b = X v_b: row r of X is column b0 + r of the block, above the diagonal;
            // four lanes per row, each over every fourth column
            const int r = tid >> 2, ph = tid & 3;
            const Cx<T>* xr = L + (int64_t)(b0 + r) * n + b0;
            Cx<T> acc[RC];
#pragma unroll
            for (int q = 0; q < RC; ++q) acc[q] = cx<T>(0, 0);
            if (r < bw)
                for (int c = ph; c < r; c += 4) {
                    const Cx<T> xv = xr[c];
#pragma unroll
                    for (int q = 0; q < RC; ++q) cfma(acc[q], xv, v[q * n + b0 + c]);
                }
#pragma unroll
            for (int q = 0; q < RC; ++q)
#pragma unroll
                for (int off = 1; off < 4; off <<= 1) {
                    acc[q].re += __shfl_xor(acc[q].re, off, 64);
                    acc[q].im += __shfl_xor(acc[q].im, off, 64);
                }
            if (ph == 0 && r < bw) {
#pragma unroll
                for (int q = 0; q < RC; ++q) xb[q][r] = v[q * n + b0 + r] + acc[q];
            }
        }
        __syncthreads();
        if (tid < bw) {
#pragma unroll
            for (int q = 0; q < RC; ++q) v[q * n + b0 + tid] = xb[q][tid];
        }
        // later rows (pivots and update rows): v_i -= L(i, block) x_b
        for (int i = b0 + bw + tid; i < n; i += TRI_NT) {
            Cx<T> acc[RC];
#pragma unroll
            for (int q = 0; q < RC; ++q) acc[q] = v[q * n + i];
            for (int c = 0; c < bw; ++c) {
                const Cx<T> lv = L[(int64_t)(b0 + c) * n + i];
#pragma unroll
                for (int q = 0; q < RC; ++q) cfms(acc[q], lv, xb[q][c]);
            }
#pragma unroll
            for (int q = 0; q < RC; ++q) v[q * n + i] = acc[q];
        }
        __syncthreads();
    }
    // x_mid = D^{-1} x_S; the update rows go to the parent's slots
    for (int i = tid; i < n; i += TRI_NT) {
        const Cx<T> dv = i < s ? A.dinv[it.start + i] : cx<T>(0, 0);
        const int pm = i < s ? 0 : A.pmap[it.pmap + i - s];
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            if (q >= nr) break;
            const int64_t rr = rhs0 + q;
            const Cx<T> y = v[q * n + i];
            if (i < s) A.xmid[rr * A.naux + it.start + i] = y * dv;
            else A.c2[rr * A.c2ld + it.push + pm] = y;
        }
    }
}

template <typename T, int RC>
__global__ __launch_bounds__(TRI_NT) void k_bwd_tri(PassArgs<T> A) {
    extern __shared__ unsigned char smem_raw[];
    Cx<T>* w = reinterpret_cast<Cx<T>*>(smem_raw);  // [RC][n]: x_mid and x_U, then x
    __shared__ Cx<T> tb[RC][64];
    if (A.run && !*A.run) return;
    const SolveItem it = A.items[blockIdx.x];
    const int n = it.n, s = it.s;
    const int rhs0 = blockIdx.y * RC;
    const int nr = min(RC, A.nrhs - rhs0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const Cx<T>* L = A.G + it.loff;
    // [x_mid; x_U] of this front; the update-set values go on to the children
    for (int i = tid; i < n; i += TRI_NT) {
        int p0 = -1, p1 = -1;
        if (i >= s) {
            if (it.cxu0 >= 0) p0 = A.cmap[it.moff + i];
            if (it.cxu1 >= 0) p1 = A.cmap[it.moff + n + i];
        }
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            Cx<T> val = cx<T>(0, 0);
            if (q < nr) {
                const int64_t rr = rhs0 + q;
                if (i < s) {
                    val = A.xmid[rr * A.naux + it.start + i];
                } else {
                    val = A.xu[rr * A.xuld + it.xu + i - s];
                    if (p0 >= 0) A.xu[rr * A.xuld + it.cxu0 + p0] = val;
                    if (p1 >= 0) A.xu[rr * A.xuld + it.cxu1 + p1] = val;
                }
            }
            w[q * n + i] = val;
        }
    }
    __syncthreads();
    // a leaf writes only its pivots on the panel's own planes: the blocks of
    // auxiliary-plane pivots before them are not needed
    const int bstop = it.leaf ? min(A.ga * (it.cellw >> 16), s) / 64 * 64 : 0;
    for (int b0 = (s - 1) / 64 * 64; b0 >= bstop; b0 -= 64) {
        const int bw = min(64, s - b0);
        // t_c = w_c - sum over the later rows i of L(i, b0 + c) x_i: one wave per
        // column, its lanes down the rows
        for (int c = wave; c < bw; c += TRI_NT / 64) {
            const Cx<T>* lc = L + (int64_t)(b0 + c) * n;
            Cx<T> acc[RC];
#pragma unroll
            for (int q = 0; q < RC; ++q) acc[q] = cx<T>(0, 0);
            for (int i = b0 + bw + lane; i < n; i += 64) {
                const Cx<T> lv = lc[i];
#pragma unroll
                for (int q = 0; q < RC; ++q) cfma(acc[q], lv, w[q * n + i]);
            }
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                acc[q].re = wave_sum(acc[q].re);
                acc[q].im = wave_sum(acc[q].im);
                if (lane == 0) tb[q][c] = w[q * n + b0 + c] - acc[q];
            }
        }
        __syncthreads();
        {   // x_b = X^T t: x_c = t_c + sum over r > c of X(r, c) t_r; four lanes per column
            const int c = tid >> 2, ph = tid & 3;
            Cx<T> acc[RC];
#pragma unroll
            for (int q = 0; q < RC; ++q) acc[q] = cx<T>(0, 0);
            if (c < bw)
                for (int r = c + 1 + ph; r < bw; r += 4) {
                    const Cx<T> xv = L[(int64_t)(b0 + r) * n + b0 + c];
#pragma unroll
                    for (int q = 0; q < RC; ++q) cfma(acc[q], xv, tb[q][r]);
                }
#pragma unroll
            for (int q = 0; q < RC; ++q)
#pragma unroll
                for (int off = 1; off < 4; off <<= 1) {
                    acc[q].re += __shfl_xor(acc[q].re, off, 64);
                    acc[q].im += __shfl_xor(acc[q].im, off, 64);
                }
            if (ph == 0 && c < bw) {
#pragma unroll
                for (int q = 0; q < RC; ++q) w[q * n + b0 + c] = tb[q][c] + acc[q];
            }
        }
        __syncthreads();
    }
    // the front's pivots: to the children's update-set values and the grid
    for (int j = bstop + tid; j < s; j += TRI_NT) {
        int o0 = -1, o1 = -1;
        if (it.cxu0 >= 0) o0 = A.cmap[it.moff + j];
        if (it.cxu1 >= 0) o1 = A.cmap[it.moff + n + j];
        const int b = pivot_box(it, A.Nx, A.NxNy, j);
        const int q3 = b / A.NxNy, lat = b - q3 * A.NxNy;
        const bool oplane = q3 >= A.ga;
        const int64_t ogi = (int64_t)(A.lo + q3 - A.ga - A.plane0) * A.NxNy + lat;
        const bool onext = A.couple && A.mode == 0 && q3 == A.nz - 1;
        const Cx<double> ocf = onext ? plane_coupling(A, lat) : cx<double>(0, 0);
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            if (q >= nr) break;
            const int64_t rr = rhs0 + q;
            const Cx<T> x = w[q * n + j];
            if (o0 >= 0) A.xu[rr * A.xuld + it.cxu0 + o0] = x;
            if (o1 >= 0) A.xu[rr * A.xuld + it.cxu1 + o1] = x;
            if (oplane) {
                Cx<double>* up = A.dst + rr * A.ld + ogi;
                const Cx<double> xd = ccast<double>(x);
                if (A.mode == 0) {
                    *up = xd;
                    if (onext) up[A.NxNy] = up[A.NxNy] - ocf * xd;
                } else {
                    *up = *up - xd;
                }
            }
        }
    }
}

template <typename T, int RC>
static void tri_rc(const PassArgs<T>& A, int nwork, int nmax, bool fwd, hipStream_t st) {
    const size_t shm = sizeof(Cx<T>) * (size_t)RC * nmax;
    const dim3 grid(nwork, (A.nrhs + RC - 1) / RC);
    if (fwd) HSW_LAUNCH((k_fwd_tri<T, RC>), grid, dim3(TRI_NT), shm, st, A);
    else HSW_LAUNCH((k_bwd_tri<T, RC>), grid, dim3(TRI_NT), shm, st, A);
}

template <typename T>
void launch_tri(const PassArgs<T>& A, int nwork, int nmax, bool fwd, hipStream_t st) {
    if (nwork <= 0) return;
    switch (solve_rhs_chunk<T>(A.nrhs, nmax)) {
        case 8: tri_rc<T, 8>(A, nwork, nmax, fwd, st); break;
        case 4: tri_rc<T, 4>(A, nwork, nmax, fwd, st); break;
        case 2: tri_rc<T, 2>(A, nwork, nmax, fwd, st); break;
        default: tri_rc<T, 1>(A, nwork, nmax, fwd, st); break;
    }
}

// ---------------------------------------------------------------------------
template <typename T, int RC, int RB, int NT>
static void fwd_rc(const PassArgs<T>& A, int nwork, int smax, hipStream_t st) {
    size_t shm = sizeof(Cx<T>) * ((size_t)RC * smax + (size_t)(NT / 64) * RB * RC);
    dim3 grid(nwork, (A.nrhs + RC - 1) / RC);
    HSW_LAUNCH((k_fwd<T, RC, RB, NT>), grid, dim3(NT), shm, st, A);
}
template <typename T, int RC, int CB, int NT>
static void bwd_rc(const PassArgs<T>& A, int nwork, int nmax, hipStream_t st) {
    size_t shm = sizeof(Cx<T>) * (size_t)RC * nmax;
    dim3 grid(nwork, (A.nrhs + RC - 1) / RC);
    HSW_LAUNCH((k_bwd<T, RC, CB, NT>), grid, dim3(NT), shm, st, A);
}

// Right-hand sides per workgroup: as many as fit 64 KiB of LDS (front vector
// plus the forward pass's reduction buffer of at most 8 waves x 64 rows), at
// most 8.
template <typename T>
int solve_rhs_chunk(int nrhs, int nmax) {
    int rc = 8;
    while (rc > 1 && (size_t)rc * (nmax + 512) * sizeof(Cx<T>) > 65536) rc >>= 1;
    while (rc > 1 && rc / 2 >= nrhs) rc >>= 1;
    return rc;
}

template <typename T, int RB, int NT>
static void fwd_cfg(const PassArgs<T>& A, int nwork, int smax, int nmax, hipStream_t st) {
    switch (solve_rhs_chunk<T>(A.nrhs, nmax)) {
        case 8: fwd_rc<T, 8, RB, NT>(A, nwork, smax, st); break;
        case 4: fwd_rc<T, 4, RB, NT>(A, nwork, smax, st); break;
        case 2: fwd_rc<T, 2, RB, NT>(A, nwork, smax, st); break;
        default: fwd_rc<T, 1, RB, NT>(A, nwork, smax, st); break;
    }
}
template <typename T, int CB, int NT>
static void bwd_cfg(const PassArgs<T>& A, int nwork, int nmax, hipStream_t st) {
    switch (solve_rhs_chunk<T>(A.nrhs, nmax)) {
        case 8: bwd_rc<T, 8, CB, NT>(A, nwork, nmax, st); break;
        case 4: bwd_rc<T, 4, CB, NT>(A, nwork, nmax, st); break;
        case 2: bwd_rc<T, 2, CB, NT>(A, nwork, nmax, st); break;
        default: bwd_rc<T, 1, CB, NT>(A, nwork, nmax, st); break;
    }
}

// Block shapes: the tables in plan.hpp, in the same order.
template <typename T, int I>
static void fwd_pick(const PassArgs<T>& A, int nwork, int cfg, int smax, int nmax, hipStream_t st) {
    if constexpr (I + 1 < N_FWD_SHAPES) {
        if (cfg != I) {
            fwd_pick<T, I + 1>(A, nwork, cfg, smax, nmax, st);
            return;
        }
    }
    fwd_cfg<T, FWD_SHAPES[I].block, FWD_SHAPES[I].threads>(A, nwork, smax, nmax, st);
}
template <typename T, int I>
static void bwd_pick(const PassArgs<T>& A, int nwork, int cfg, int nmax, hipStream_t st) {
    if constexpr (I + 1 < N_BWD_SHAPES) {
        if (cfg != I) {
            bwd_pick<T, I + 1>(A, nwork, cfg, nmax, st);
            return;
        }
    }
    bwd_cfg<T, BWD_SHAPES[I].block, BWD_SHAPES[I].threads>(A, nwork, nmax, st);
}
template <typename T>
void launch_fwd(const PassArgs<T>& A, int nwork, int cfg, int smax, int nmax, hipStream_t st) {
    if (nwork <= 0) return;
    fwd_pick<T, 0>(A, nwork, cfg, smax, nmax, st);
}
template <typename T>
void launch_bwd(const PassArgs<T>& A, int nwork, int cfg, int nmax, hipStream_t st) {
    if (nwork <= 0) return;
    bwd_pick<T, 0>(A, nwork, cfg, nmax, st);
}

template <typename T>
void launch_rhs_scatter(const PassArgs<T>& A, hipStream_t st) {
    if (A.naux <= 0) return;
    const dim3 grid((A.naux + 63) / 64, (A.nrhs + 15) / 16);
    HSW_LAUNCH(k_rhs_scatter<T>, grid, dim3(256), 0, st, A);
}
// Forms of the forward matrix-core pass: 0 / 3: 64 rows per workgroup, 4 /
// 8 waves splitting the contraction; 1 / 4: 16 rows, 4 / 8 waves; 2:
// row-split (64 rows, needs fwd_rs_lds_bytes(smax) of LDS); 5: 64 rows with
// each item's contraction split over A.nsplit workgroups, then a finishing
// launch (A.part holds the partial blocks).
template <typename T>
void launch_fwd_mm(const PassArgs<T>& A, int nwork, int form, int smax, hipStream_t st) {
    if (nwork <= 0) return;
    const dim3 grid(nwork, (A.nrhs + 15) / 16);
    constexpr int FP = sizeof(T) == 4 ? 4 : 2;
    switch (form) {
    case 0: HSW_LAUNCH((k_fwd_mm<T, 4, 4>), grid, dim3(256), 0, st, A); break;
    case 1: HSW_LAUNCH((k_fwd_mm<T, 1, 4>), grid, dim3(256), 0, st, A); break;
    case 2: HSW_LAUNCH((k_fwd_rs<T, FP>), grid, dim3(256), fwd_rs_lds_bytes<T>(smax), st, A); break;
    case 3: HSW_LAUNCH((k_fwd_mm<T, 4, 8>), grid, dim3(512), 0, st, A); break;
    case 4: HSW_LAUNCH((k_fwd_mm<T, 1, 8>), grid, dim3(512), 0, st, A); break;
    case 7: HSW_LAUNCH((k_fwd_mm<T, 1, 2>), grid, dim3(128), 0, st, A); break;
    case 6: {
        const dim3 gs(nwork * A.nsplit, grid.y);
        HSW_LAUNCH((k_fwd_mm<T, 1, 4, 1>), gs, dim3(256), 0, st, A);
        HSW_LAUNCH((k_fwd_fin<T, 1>), grid, dim3(256), 0, st, A);
        break;
    }
    default: {
        const dim3 gs(nwork * A.nsplit, grid.y);
        HSW_LAUNCH((k_fwd_mm<T, 4, 4, 1>), gs, dim3(256), 0, st, A);
        HSW_LAUNCH((k_fwd_fin<T, 4>), grid, dim3(256), 0, st, A);
    }
    }
}
// Forms of the backward matrix-core pass: 0: 64 columns per workgroup, 4
// waves; 1 / 2 / 3: 16 columns, 4 / 8 / 16 waves (complex128: 8 at most,
// for registers); 4: 64 columns with each item's contraction split over
// A.nsplit workgroups, then a finishing launch; 5 / 6: as 1 / 2 with four
// chunks in flight per wave (two in the others).
template <typename T>
void launch_bwd_mm(const PassArgs<T>& A, int nwork, int form, hipStream_t st) {
    if (nwork <= 0) return;
    const dim3 grid(nwork, (A.nrhs + 15) / 16);
    constexpr int W16 = sizeof(T) == 4 ? 16 : 8;
    switch (form) {
    case 0: HSW_LAUNCH((k_bwd_mm<T, 4, 4>), grid, dim3(256), 0, st, A); break;
    case 1: HSW_LAUNCH((k_bwd_mm<T, 1, 4>), grid, dim3(256), 0, st, A); break;
    case 2: HSW_LAUNCH((k_bwd_mm<T, 1, 8>), grid, dim3(512), 0, st, A); break;
    case 3: HSW_LAUNCH((k_bwd_mm<T, 1, W16>), grid, dim3(64 * W16), 0, st, A); break;
    case 4: {
        const dim3 gs(nwork * A.nsplit, grid.y);
        HSW_LAUNCH((k_bwd_mm<T, 4, 4, 1>), gs, dim3(256), 0, st, A);
        HSW_LAUNCH((k_bwd_fin<T, 4>), grid, dim3(256), 0, st, A);
        break;
    }
    case 8: HSW_LAUNCH((k_bwd_mm<T, 1, 2>), grid, dim3(128), 0, st, A); break;
    case 7: {
        const dim3 gs(nwork * A.nsplit, grid.y);
        HSW_LAUNCH((k_bwd_mm<T, 1, 4, 1>), gs, dim3(256), 0, st, A);
        HSW_LAUNCH((k_bwd_fin<T, 1>), grid, dim3(256), 0, st, A);
        break;
    }
    case 5: HSW_LAUNCH((k_bwd_mm<T, 1, 4, 0, 4>), grid, dim3(256), 0, st, A); break;
    default: HSW_LAUNCH((k_bwd_mm<T, 1, 8, 0, 4>), grid, dim3(512), 0, st, A); break;
    }
}

#define HSW_INST(T)                                                                          \
    template void launch_tri<T>(const PassArgs<T>&, int, int, bool, hipStream_t);           \
    template void launch_fwd<T>(const PassArgs<T>&, int, int, int, int, hipStream_t);       \
    template void launch_bwd<T>(const PassArgs<T>&, int, int, int, hipStream_t);            \
    template void launch_fwd_mm<T>(const PassArgs<T>&, int, int, int, hipStream_t);         \
    template size_t fwd_rs_lds_bytes<T>(int);                                                \
    template void launch_rhs_scatter<T>(const PassArgs<T>&, hipStream_t);                    \
    template void launch_bwd_mm<T>(const PassArgs<T>&, int, int, hipStream_t);              \
    template int solve_rhs_chunk<T>(int, int);
HSW_INST(float)
HSW_INST(double)
#undef HSW_INST

}  // namespace hsw
