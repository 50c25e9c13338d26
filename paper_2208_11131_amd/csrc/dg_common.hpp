// dg_common.hpp -- plain structs shared by the host runtime and the HIP
// kernels of the DG library (argument blocks and per-order tables).
#pragma once
#include <stdint.h>

namespace dgk {

constexpr int MAXP = 8;     // highest order (modes / Gauss points per axis)
constexpr int MAXF = 9;     // a point's values: stored fields (dim+2, +1 tracer or AV) plus dim forcing components

// Per-order 1D tables on the p Gauss-Legendre nodes x_j of [-1, 1]
// (Sec. 2.3 scaled Legendre basis, Sec. 2.4 quadrature, Sec. 3.2 recovery).
template <typename T>
struct Tab {
    T B[MAXP][MAXP];    // B[l][j]  = Pt_l(x_j)              modal -> point
    T Bd[MAXP][MAXP];   // Bd[l][j] = Pt_l'(x_j)             modal -> point derivative
    T D[MAXP][MAXP];    // D[j][k]  = L_k'(x_j)              collocation derivative
    T g[MAXP];          // Gauss weights
    T Lp[MAXP];         // L_j(+1)  Lagrange basis of the nodes at the upper end
    T Lm[MAXP];         // L_j(-1)
    T ep[MAXP];         // Pt_m(+1)
    T em[MAXP];         // Pt_m(-1)
    T rvL[MAXP];        // recovered face value   = sum_m rvL[m] wL_m + rvR[m] wR_m
    T rvR[MAXP];        //   (normal mode index m, per transverse mode)
    T rdL[MAXP];        // recovered d/dxi* at the face (scale by 1/(f h))
    T rdR[MAXP];
    // total-degree basis P_n: the same four vectors for the lines of
    // transverse degree tau (data of normal degree <= n - tau, recovered to
    // normal degree n + 1 - tau), indexed [tau][m]
    T prvL[MAXP][MAXP];
    T prvR[MAXP][MAXP];
    T prdL[MAXP][MAXP];
    T prdR[MAXP][MAXP];
};

// Physics and discretisation constants of one context (FP64; kernels convert).
struct Phys {
    double gamma, nu, kappa, h;
    double two_over_h;   // 2/h: d/dx = (2/h) d/dxi
    double inv_fh;       // 1/(f h): d/dx = (1/(f h)) d/dxi* on the recovery domain
    double pref;         // 2^(1-d)/h: prefactor of volume and surface sums
    double half_h;       // h/2: converts a source projection to the common prefactor
    int ns_on;           // nu > 0, kappa > 0 or a diffusing tracer (eta > 0)
    int av_on;           // AV field present
    double av_scale, f_v, sink;   // sink = p/(f_tau h): alpha/tau = alpha c_s sink
    double f_w, s_thr, alpha_max, eps_fac;   // s_thr = s_onset/p^2, eps_fac = h/p
    int order;           // p
    double eta;          // passive-tracer diffusivity (Sec. 3.4)
};

// Mesh geometry.  Face space of direction a has nf[a] planes along a
// (n[a] periodic, n[a]+1 with closed ends) and n[b] along the other axes.
struct Geo {
    int n[3];
    int nf[3];
    int bc[3];
    long long ncells;
    long long nfaces[3];
    long long fb_off[3];   // element offset of direction a's block in the face buffer
};

// Volume/stage kernel.  out = c_base*base + c_cur*cur + c_L*dt*L(cur);
// optionally out2 = d_x2*x2 + d_cur*cur + d_L*dt*L(cur) (5-stage RK, stage 4).
struct VolArgs {
    const double *cur;
    const double *base;
    const double *x2;
    double *out;
    double *out2;
    double c_base, c_cur, c_L, d_x2, d_cur, d_L;
    const double *dt_ptr;   // device dt (used when not null)
    double dt;
    const void *fb;         // face fluxes (T), weighted by the transverse Gauss weights
    const void *forcing;    // driving field at the Gauss points [cell][dim][p^d] (T) or null
    const double *R_prev;   // [cell] dlnS/dt of the previous step (AV) or null
    double *R_out;          // [cell] dlnS/dt of `cur` (stage 1) or null
    int *flag;              // error flag: 1 non-physical mean, 2 non-finite
    int check;              // test the new cell means (RK stages) or not (RHS)
    int cells_per_block;
};

struct FaceArgs {
    const double *w;
    void *fb;
    int faces_per_block;
    // CFL finalize folded into this launch (cfl_part != null): block (0, 0)
    // reduces the CFL kernel's per-block maxima and writes dt
    const double *cfl_part;
    double *cfl_res;       // [0] dt, [1] c_max, [2] v_max
    double *cfl_dt_copy;   // optional second copy of dt
    double cfl_num;        // f_CFL h / (2 p)
    int cfl_nblk;
};

struct CflArgs {
    const double *w;
    double *part;          // [block][2]: c_s max, |v| max of each block
    int cells_per_block;
};

// One box of a batched ensemble (device table, one entry per box of a
// (dim, order) group).  reg[0] is the caller's state, reg[1..3] the RK
// registers; start[k] = first flat block of this box in the grouped launch of
// kind k (0 volume, 1 face, 2 CFL).
struct BoxDesc {
    Phys ph;
    Geo geo;
    double *reg[4];
    void *fb;
    double *cfl_part;
    double *dt;          // [0] dt, [1] c_max, [2] v_max of the box
    int *flag;
    long long start[3];
    long long nblocks[3];
    int cells_per_block, faces_per_block, cfl_cells;
    int bidx;            // index of the box in its batch
};

// RK stage of a grouped launch: register roles (-1 = none) and Shu-Osher
// coefficients, shared by every box of the group (same order, same scheme).
struct StageDesc {
    int cur, base, x2, out, out2;
    double c_base, c_cur, c_L, d_x2, d_cur, d_L;
};

// Launch grid of the single-box face kernels: bricks of C cells per axis,
// ceil(nf[a] / C) along axis a, each with dim C^(dim-1) pencil blocks (all
// directions); grid.x = those blocks times the bricks along x, grid.y and
// grid.z the bricks along y and z.
inline void face_grid(const Geo &g, int dim, int C, long long &gx, long long &gy, long long &gz)
{
    const long long k1 = dim == 3 ? (long long)C * C : C;
    gx = dim * k1 * ((g.nf[0] + C - 1) / C);
    gy = (g.nf[1] + C - 1) / C;
    gz = dim == 3 ? (g.nf[2] + C - 1) / C : 1;
}

}  // namespace dgk
