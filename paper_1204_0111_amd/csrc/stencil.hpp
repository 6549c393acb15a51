// Entries of the stretched 7-point operator, generated on the fly.
//
// With node stretches e_j, inverse half-node stretches ie_j^{+-} = 1/e_j(x_j +- h/2),
// P_j = e_k e_l (the two other axes) and E = e1 e2 e3:
//   (H u)_p = h^-2 sum_j [ P_j (ie_j^+ + ie_j^-) u_p - P_j ie_j^+ u_{p+e_j}
//                          - P_j ie_j^- u_{p-e_j} ] - kappa^2 E u_p / c(p)^2,
// the symmetric form of the stretched Laplacian (Sec. 1, Eq. 1.1 discretised
// with the complex-stretched PML; complex symmetric as Sec. 1.1 requires).
// kappa^2 = omega^2 for A and (omega + i alpha)^2 for J (Sec. 1.1, Eq. 1.5).
// Entries are formed in FP64 whatever the working precision.
#pragma once

#include "devtypes.hpp"

namespace hsw {

struct NodeStretch {
    Cx<double> e[3];     // node stretch per axis
    Cx<double> im[3];    // inverse half-node stretch below (x_j - h/2)
    Cx<double> ip[3];    // inverse half-node stretch above (x_j + h/2)
};

// Velocity at padded node (a1, a2, g3) (g3 = global padded plane), clamped
// to the nearest interior node.
__device__ inline double velocity_at(const ProbDev& Q, int a1, int a2, int g3) {
    int i1 = min(max(a1 - Q.gamma, 0), Q.n[0] - 1);
    int i2 = min(max(a2 - Q.gamma, 0), Q.n[1] - 1);
    int i3 = min(max(g3 - Q.gamma, 0), Q.n[2] - 1);
    return Q.c[(int64_t)i1 + (int64_t)Q.n[0] * (i2 + (int64_t)Q.n[1] * i3)];
}

// Lateral stretches from the problem's tables; x3 from (e3, ie3) tables
// given by the caller (physical or a panel's artificial ones), node index q.
__device__ inline NodeStretch node_stretch(const ProbDev& Q, const Cx<double>* et, int a1, int a2,
                                           const Cx<double>* e3n, const Cx<double>* ie3h, int q) {
    NodeStretch s;
    const Cx<double>* t1 = et + Q.e_off[0];
    const Cx<double>* t2 = et + Q.e_off[1];
    s.e[0] = t1[a1];
    s.im[0] = t1[Q.N[0] + a1];
    s.ip[0] = t1[Q.N[0] + a1 + 1];
    s.e[1] = t2[a2];
    s.im[1] = t2[Q.N[1] + a2];
    s.ip[1] = t2[Q.N[1] + a2 + 1];
    s.e[2] = e3n[q];
    s.im[2] = ie3h[q];
    s.ip[2] = ie3h[q + 1];
    return s;
}

__device__ inline Cx<double> axis_weight(const NodeStretch& s, int j) {
    // P_j = product of the node stretches of the two other axes
    return j == 0 ? s.e[1] * s.e[2] : (j == 1 ? s.e[0] * s.e[2] : s.e[0] * s.e[1]);
}

__device__ inline Cx<double> diag_entry(const NodeStretch& s, double c, Cx<double> kappa2,
                                        double inv_h2) {
    Cx<double> E = (s.e[0] * s.e[1]) * s.e[2];
    Cx<double> d = scale(kappa2 * E, -1.0 / (c * c));
    for (int j = 0; j < 3; ++j) {
        Cx<double> P = axis_weight(s, j);
        d = d + scale(P * (s.ip[j] + s.im[j]), inv_h2);
    }
    return d;
}

// Coupling between a node (a1, a2, q) and its upper neighbour along axis ax:
// -P_ax ie_ax^+ / h^2, from the two other axes' node stretches and the
// inverse half-node stretch above the node along ax.  The three table entries
// are picked by pointer, so nothing is indexed at run time (a run-time index
// into a local array would be placed in scratch memory).
__device__ inline Cx<double> coupling_entry(const ProbDev& Q, const Cx<double>* et,
                                            const Cx<double>* e3n, const Cx<double>* ie3h, int a1,
                                            int a2, int q, int ax, double inv_h2) {
    const Cx<double>* t1 = et + Q.e_off[0];
    const Cx<double>* t2 = et + Q.e_off[1];
    const Cx<double>* pa = ax == 0 ? t2 + a2 : t1 + a1;
    const Cx<double>* pb = ax == 2 ? t2 + a2 : e3n + q;
    const Cx<double>* pc = ax == 0 ? t1 + Q.N[0] + a1 + 1
                                   : (ax == 1 ? t2 + Q.N[1] + a2 + 1 : ie3h + q + 1);
    return scale((*pa * *pb) * *pc, -inv_h2);
}

__device__ inline Cx<double> kappa_sq(const ProbDev& Q, double alpha) {
    return cx<double>(Q.omega * Q.omega - alpha * alpha, 2.0 * Q.omega * alpha);
}

}  // namespace hsw
