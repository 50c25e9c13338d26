// dg_kernels.hpp -- HIP kernels of the DG right-hand side for gfx950.
//
// Included once by each instantiation unit (dg_inst_*.hip).  Each unit gets
// its own copy of the per-order tables in __constant__ memory (uploaded by
// the host runtime through the unit's dgk_upload_* entry).
//
// Work decomposition (one HIP thread block = a tile of whole cells or a pencil
// of faces; intermediates in LDS, the state read from and written to HBM by
// the passes that need it):
//   face kernel    a pencil of faces of one direction (blocks in brick-major
//                  order, all directions of a brick together): traces of
//                  both cells (normal lines read from HBM), HLLC, and
//                  (viscous/AV) the interface recovery of Sec. 3.2 with the
//                  Navier-Stokes/AV flux; one single-valued flux per face
//                  point to the face buffer.
//   volume kernel  per cell: modal -> Gauss-point values by sum factorisation
//                  (one p x p operator per axis, the first reading HBM),
//                  collocation gradients, point fluxes and sources, D^T fused
//                  with the face lift in point space, point -> modal
//                  projection whose last pass is fused with the FP64 SSP-RK
//                  stage combination (prefactor 2^(1-d)/h) and write-back.
//   cfl kernel     maxima of c_s and |v| over all volume Gauss points.
// Fixed-tile variants (tile and forcing as template parameters) exist for
// the tuned tiles; every variant rounds identically (contraction is limited
// to single expressions by the build).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "dg_common.hpp"
#include "dg_tiles.hpp"

namespace dgk {

static __constant__ Tab<double> c_tabd[MAXP + 1];
static __constant__ Tab<float> c_tabf[MAXP + 1];

template <typename T>
struct TabSel;
template <>
struct TabSel<double> {
    static __device__ __forceinline__ const Tab<double> &get(int P) { return c_tabd[P]; }
};
template <>
struct TabSel<float> {
    static __device__ __forceinline__ const Tab<float> &get(int P) { return c_tabf[P]; }
};

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// max that propagates NaN (order independent)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

enum { M_B = 0, M_BT = 1, M_D = 2, M_DT = 3, M_BD = 4 };

// Entry (k, i) of the operator of a line pass: out_i = sum_k M(k, i) in_k.
template <int P, typename T, int MAT>
__device__ __forceinline__ T mat(int k, int i)
{
    const Tab<T> &t = TabSel<T>::get(P);
    if (MAT == M_B) return t.B[k][i];        // point i from mode k
    if (MAT == M_BT) return t.B[i][k];       // mode i from point k
    if (MAT == M_D) return t.D[i][k];        // derivative at point i
    if (MAT == M_DT) return t.D[k][i];       // transpose of the derivative
    return t.Bd[k][i];                       // derivative of mode k at point i
}

// Padded point layout of one per-cell array: rows along x hold PP entries
// (PP = p + 1 for even p, p for odd p), so that the lines of a pass along any
// axis fall into different LDS banks.  Point j = j_x + p (j_y + p j_z) lives
// at j_x + PP (j_y + p j_z); an array takes NAP = PP p^(d-1) entries.
template <int P>
struct Pad {
    static constexpr int PP = (P % 2 == 0) ? P + 1 : P;
};

// Row pitch of the face kernel's arrays: unpadded at p = 4, where that
// measured faster (the face kernel's lines are short and its LDS footprint
// per pencil sets the occupancy), padded like the volume kernel otherwise.
template <int P>
struct FacePad {
    static constexpr int PP = (P == 4) ? P : Pad<P>::PP;
};

// Position of point j in a per-cell array with row pitch RP.
template <int P, int RP = Pad<P>::PP>
__device__ __forceinline__ int ppos(int j)
{
    return (j % P) + RP * (j / P);
}

// line_pass over narr contiguous padded arrays of (d-dimensional) points.
// Each thread takes two lines per iteration (q and q + blockDim) and issues
// the loads of both before their FMAs, so that two LDS round trips overlap.
template <int P, int DA, int AX, int RP = Pad<P>::PP>
__device__ __forceinline__ int pad_line_offset(int q)
{
    constexpr int PP = RP;
    constexpr int NAP = PP * ipow(P, DA - 1);
    if (AX == 0) return q * PP;
    if (AX == 1) return (q / P) * (PP * P) + (q % P);
    const int a = q / (P * P), t = q - a * (P * P);
    return a * NAP + (t % P) + PP * (t / P);
}

template <int P, int DA, int AX, typename T, int MAT, bool ACC, int NTC = 0, int RP = Pad<P>::PP>
__device__ __forceinline__ void line_pass_pad(const T *__restrict__ in, T *__restrict__ out, int narr)
{
    constexpr int PP = RP;
    constexpr int NL = ipow(P, DA - 1);                  // lines per array
    constexpr int S = (AX == 0) ? 1 : (AX == 1 ? PP : PP * P);
    const int nitems = narr * NL;
    const int nt = NTC > 0 ? NTC : (int)blockDim.x;      // NTC: block size fixed at compile time
    // rounds of 2 nt lines (two per thread) while the block has that many,
    // then at most one round of single lines; the choice is uniform
    for (int b0 = 0; b0 < nitems; b0 += 2 * nt) {
        const int q = b0 + threadIdx.x;
        if (b0 + nt < nitems) {
            const bool two = q + nt < nitems;
            const int o0 = pad_line_offset<P, DA, AX, RP>(q);
            const int o1 = two ? pad_line_offset<P, DA, AX, RP>(q + nt) : o0;
            T x0[P], x1[P], y0[P], y1[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                x0[k] = in[o0 + k * S];
                x1[k] = in[o1 + k * S];
            }
            if (ACC) {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    y0[i] = out[o0 + i * S];
                    y1[i] = out[o1 + i * S];
                }
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
                T a0 = ACC ? y0[i] : T(0), a1 = ACC ? y1[i] : T(0);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const T m = mat<P, T, MAT>(k, i);
                    a0 = fma(m, x0[k], a0);
                    a1 = fma(m, x1[k], a1);
                }
                y0[i] = a0;
                y1[i] = a1;
            }
#pragma unroll
            for (int i = 0; i < P; ++i) out[o0 + i * S] = y0[i];
            if (two) {
#pragma unroll
                for (int i = 0; i < P; ++i) out[o1 + i * S] = y1[i];
            }
        } else if (q < nitems) {
            const int o0 = pad_line_offset<P, DA, AX, RP>(q);
            T x0[P], y0[P];
#pragma unroll
            for (int k = 0; k < P; ++k) x0[k] = in[o0 + k * S];
            if (ACC) {
#pragma unroll
                for (int i = 0; i < P; ++i) y0[i] = out[o0 + i * S];
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
                T a0 = ACC ? y0[i] : T(0);
#pragma unroll
                for (int k = 0; k < P; ++k) a0 = fma(mat<P, T, MAT>(k, i), x0[k], a0);
                y0[i] = a0;
            }
#pragma unroll
            for (int i = 0; i < P; ++i) out[o0 + i * S] = y0[i];
        }
    }
}

// VW consecutive doubles moved by one global access (VW = 2: 16-byte loads
// and stores; the state arrays are 16-byte aligned and a group never
// straddles a field or a cell when the per-cell length is even).
template <int VW>
struct DV {
    double x[VW];
};

template <int VW>
__device__ __forceinline__ DV<VW> ldv(const double *p)
{
    DV<VW> r;
    if constexpr (VW == 2) {
        const double2 t = *(const double2 *)p;
        r.x[0] = t.x;
        r.x[1] = t.y;
    } else {
        r.x[0] = *p;
    }
    return r;
}

template <int VW>
__device__ __forceinline__ void stv(double *p, const DV<VW> &v)
{
    if constexpr (VW == 2)
        *(double2 *)p = make_double2(v.x[0], v.x[1]);
    else
        *p = v.x[0];
}

template <int VW>
__device__ __forceinline__ DV<VW> zdv()
{
    DV<VW> r;
#pragma unroll
    for (int h = 0; h < VW; ++h) r.x[h] = 0.0;
    return r;
}

// D^T pass along AX accumulated into out, fused with the surface lift of the
// same lines: out_i += sum_k D(k, i) in_k + L_i(-1) Fl - L_i(+1) Fu, where
// (Fl, Fu) = lf[r] are the lower / upper face fluxes of line r of this thread
// (line q = threadIdx.x + r NTC; the block size NTC is fixed).
template <int P, int DA, int AX, typename T, int NTC, int NR>
__device__ __forceinline__ void dt_lift_pass(const T *__restrict__ in, T *__restrict__ out, int nitems,
                                             const T (*lf)[2])
{
    constexpr int PP = Pad<P>::PP;
    constexpr int S = (AX == 0) ? 1 : (AX == 1 ? PP : PP * P);
    const Tab<T> &tb = TabSel<T>::get(P);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int q = threadIdx.x + r * NTC;
        if (q < nitems) {
            const int o = pad_line_offset<P, DA, AX>(q);
            T x[P], y[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                x[k] = in[o + k * S];
                y[k] = out[o + k * S];
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
                T acc = y[i];
#pragma unroll
                for (int k = 0; k < P; ++k) acc = fma(mat<P, T, M_DT>(k, i), x[k], acc);
                out[o + i * S] = acc + (tb.Lm[i] * lf[r][0] - tb.Lp[i] * lf[r][1]);
            }
        }
    }
}

// Fields per physics variant: PH = 0 Euler, 1 Navier-Stokes, 2 artificial
// viscosity (alpha field; Navier-Stokes terms switched at run time),
// 3 Navier-Stokes with the passive tracer c rho (Sec. 3.4); PH = 4..7 are
// the same four on the total-degree basis P_n (Sec. 2.3).  Fc conserved
// fields carry face fluxes: the D + 2 hydro fields and the tracer.
template <int D, int PH>
struct Fld {
    static constexpr bool PN = PH >= 4;
    static constexpr int BASE = PN ? PH - 4 : PH;
    static constexpr int NH = D + 2;
    static constexpr bool TR = BASE == 3;
    static constexpr bool AV = BASE == 2;
    static constexpr int Fc = NH + (TR ? 1 : 0);
    static constexpr int F = Fc + (AV ? 1 : 0);
    static constexpr bool GRAD = BASE > 0;
    static constexpr bool NS = BASE == 1 || BASE == 3;   // Navier-Stokes terms compiled in
};

// Storage of one field's modal weights.  Q_n: the p^d tensor modes, index
// l_x + p (l_y + p l_z).  P_n: the modes of total degree <= n = p - 1 in the
// order l_z, l_y, l_x ascending (l_x fastest): the "line" of transverse
// digits (l_y, l_z) holds l_x = 0 .. n - l_y - l_z contiguously from
// off(l_y, l_z) = Tet(p) - Tet(p - l_z) + l_y (p - l_z) - l_y (l_y - 1)/2,
// Tet(q) = q (q+1) (q+2) / 6.  Kernels expand a cell to the tensor layout in
// registers / LDS (absent modes are 0) and store back only the P_n modes.
template <int D, int P, bool PN>
struct Basis {
    static constexpr int NM = PN ? (D == 2 ? P * (P + 1) / 2 : P * (P + 1) * (P + 2) / 6) : ipow(P, D);
    static __host__ __device__ constexpr int tet(int q) { return q * (q + 1) * (q + 2) / 6; }
    // start and length of the l_x line with transverse digits (ly, lz)
    static __device__ __forceinline__ int off(int ly, int lz)
    {
        return PN ? tet(P) - tet(P - lz) + ly * (P - lz) - ly * (ly - 1) / 2 : (ly + P * lz) * P;
    }
    static __device__ __forceinline__ int len(int ly, int lz) { return PN ? (P - ly - lz > 0 ? P - ly - lz : 0) : P; }
    // storage index of mode (lx, ly, lz), -1 if it is not in the basis
    static __device__ __forceinline__ int idx(int lx, int ly, int lz)
    {
        return (PN && lx + ly + lz > P - 1) ? -1 : off(ly, lz) + lx;
    }
};

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8);
// map them so that each XCD works on one contiguous range of logical blocks
// (neighbouring tiles then share that XCD's L2).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned q = nb / 8, r = nb % 8;
    const unsigned x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// point physics (Sec. 2 eq. flux_matrix, Sec. 3.3, Sec. 4.1)
// ---------------------------------------------------------------------------

template <int D, typename T>
struct Prim {
    T rho, ir, v[D], p;
};

template <int D, typename T>
__device__ __forceinline__ Prim<D, T> primitives(const T *u, T gamma)
{
    Prim<D, T> s;
    s.rho = u[0];
    s.ir = T(1) / s.rho;
    T v2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        s.v[i] = u[1 + i] * s.ir;
        v2 += s.v[i] * s.v[i];
    }
    s.p = (gamma - T(1)) * (u[D + 1] - T(0.5) * s.rho * v2);
    return s;
}

// Euler flux along axis a: (m_a, m_a v + p e_a, (e + p) v_a).
template <int D, typename T>
__device__ __forceinline__ void euler_flux(const T *u, const Prim<D, T> &s, int a, T *f)
{
    f[0] = u[1 + a];
#pragma unroll
    for (int i = 0; i < D; ++i) f[1 + i] = u[1 + a] * s.v[i] + (i == a ? s.p : T(0));
    f[D + 1] = (u[D + 1] + s.p) * s.v[a];
}

// HLLC flux (Toro ch. 10) with Davis wave-speed bounds, for NC conserved
// fields: the hydro fields and (NC = D + 3) a passive scalar c rho, whose
// flux is c rho v_a and whose star state is c_K times the star density.
template <int D, typename T, int NC = D + 2>
__device__ __forceinline__ void hllc(const T *uL, const T *uR, int a, T gamma, T *F)
{
    const Prim<D, T> L = primitives<D, T>(uL, gamma);
    const Prim<D, T> R = primitives<D, T>(uR, gamma);
    const T cL = sqrt(gamma * L.p * L.ir), cR = sqrt(gamma * R.p * R.ir);
    const T unL = L.v[a], unR = R.v[a];
    const T SL = fmin(unL - cL, unR - cR);
    const T SR = fmax(unL + cL, unR + cR);
    if (T(0) <= SL) {
        euler_flux<D, T>(uL, L, a, F);
        if (NC > D + 2) F[D + 2] = uL[D + 2] * L.v[a];
        return;
    }
    if (SR <= T(0)) {
        euler_flux<D, T>(uR, R, a, F);
        if (NC > D + 2) F[D + 2] = uR[D + 2] * R.v[a];
        return;
    }
    const T Ss = (R.p - L.p + L.rho * unL * (SL - unL) - R.rho * unR * (SR - unR)) /
                 (L.rho * (SL - unL) - R.rho * (SR - unR));
    const bool left = Ss >= T(0);
    const T *u = left ? uL : uR;
    const Prim<D, T> &K = left ? L : R;
    const T S = left ? SL : SR;
    const T un = K.v[a];
    euler_flux<D, T>(u, K, a, F);
    if (NC > D + 2) F[D + 2] = u[D + 2] * K.v[a];
    const T fac = K.rho * (S - un) / (S - Ss);
    T us[NC];
    us[0] = fac;
#pragma unroll
    for (int i = 0; i < D; ++i) us[1 + i] = (i == a) ? fac * Ss : fac * K.v[i];
    us[D + 1] = fac * (u[D + 1] * K.ir + (Ss - un) * (Ss + K.p / (K.rho * (S - un))));
    if (NC > D + 2) us[D + 2] = fac * (u[D + 2] * K.ir);
#pragma unroll
    for (int k = 0; k < NC; ++k) F[k] += S * (us[k] - u[k]);
}

// Navier-Stokes flux (added with a minus sign to the Euler flux), Sec. 3.3:
// along axis a, (0, Pi_{.a}, v.Pi_{.a} + chi (gamma-1) rho d_a e_int) with
// Pi = nu rho (grad v + grad v^T - 2/3 div v I) and primitive gradients from
// conserved ones.  g[b][f] = d u_f / d x_b.  The velocity-gradient tensor,
// its divergence and grad e_int are formed once per point (NsGrad) and
// shared by every direction.
template <int D, typename T>
struct NsGrad {
    T dv[D][D];   // dv[i][b] = d v_i / d x_b
    T div;
    T de[D];      // d e_int / d x_b
};

template <int D, typename T>
__device__ __forceinline__ NsGrad<D, T> ns_grad(const T *u, const Prim<D, T> &s, const T (*g)[MAXF])
{
    NsGrad<D, T> n;
#pragma unroll
    for (int b = 0; b < D; ++b)
#pragma unroll
        for (int i = 0; i < D; ++i) n.dv[i][b] = (g[b][1 + i] - s.v[i] * g[b][0]) * s.ir;
    n.div = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) n.div += n.dv[i][i];
    const T eps = u[D + 1] * s.ir;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        T de = (g[b][D + 1] - eps * g[b][0]) * s.ir;
#pragma unroll
        for (int i = 0; i < D; ++i) de -= s.v[i] * n.dv[i][b];
        n.de[b] = de;
    }
    return n;
}

template <int D, typename T>
__device__ __forceinline__ void ns_flux(const Prim<D, T> &s, const NsGrad<D, T> &n, int a, T gamma, T nu, T chi,
                                        T *fv)
{
    const T nr = nu * s.rho;
    fv[0] = T(0);
    T vp = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const T pi = nr * (n.dv[i][a] + n.dv[a][i] - (i == a ? T(2.0 / 3.0) * n.div : T(0)));
        fv[1 + i] = pi;
        vp += s.v[i] * pi;
    }
    fv[D + 1] = vp + chi * (gamma - T(1)) * s.rho * n.de[a];
}

template <typename T>
__device__ __forceinline__ T clamp_alpha(T al, T amax)
{
    return al < T(0) ? T(0) : (al > amax ? amax : al);
}

// ---------------------------------------------------------------------------
// face kernel
// ---------------------------------------------------------------------------
//
// One block computes a pencil of C consecutive faces of direction AX (fixed
// transverse coordinates).  It loads the C + 1 cells that these faces
// separate once, so every cell is read about once per direction.

// CC, NTC: faces per pencil and threads per block fixed at compile time (0 =
// taken from the launch); same results either way.  The pencil: faces
// a0 .. a0 + C - 1 along AX at the transverse cell coordinates cin[b != AX].
template <int D, int P, int AX, typename T, int PH, int CC = 0, int NTC = 0>
__device__ __forceinline__ void face_body(const Phys &ph, const Geo &geo, const FaceArgs &a, unsigned char *smem,
                                          const int *cin, int a0)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;          // face points (and transverse modes)
    constexpr int Fc = Fld<D, PH>::Fc;
    constexpr int F = Fld<D, PH>::F;
    constexpr bool GRAD = Fld<D, PH>::GRAD;
    constexpr bool PN = Fld<D, PH>::PN;
    using BS = Basis<D, P, PN>;
    constexpr int NM = BS::NM;         // stored modes per field
    constexpr int FNP = F * NM;        // stored weights per cell
    constexpr int NA = GRAD ? 4 : 2;
    constexpr int S = ipow(P, AX);
    constexpr int PP = FacePad<P>::PP;
    constexpr int NAP = PP * NP / P;                      // padded cell array
    constexpr int NAF = (D == 3) ? PP * P : PP;           // padded face array
    constexpr int SP = (AX == 0) ? 1 : (AX == 1 ? PP : PP * P);   // padded stride along AX
    const int C = CC > 0 ? CC : a.faces_per_block;
    const int tid = threadIdx.x, nt = NTC > 0 ? NTC : (int)blockDim.x;
    const int Q = C * F * NAF;
    const int na = geo.n[AX], nfa = geo.nf[AX];
    const int nface = min(C, nfa - a0);
    int co[3] = {cin[0], cin[1], cin[2]};
    co[AX] = 0;

    long long *cellidx = (long long *)smem;               // [C+1]
    int *mir = (int *)(cellidx + (C + 1));                // [C+1]
    // LDS: the scratch Sx of the transverse passes (5 Q entries; during the
    // normal contraction it holds the upper cells' recovery partial sums),
    // then the contraction results A (NA Q entries).  The cells themselves
    // are read straight from HBM by the normal contraction.
    T *Sx = (T *)(smem + (((C + 1) * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16);   // [5][C][F][NAF]
    T *A = Sx + 5 * Q;                                    // [NA][C][F][NAF]
    // P_n with gradients: the recovery vectors of every transverse degree,
    // [vL, dL, vR, dR][tau][m], copied to LDS (each lane of the contraction
    // indexes them by its own line's degree)
    T *rt = A + NA * Q;
    if constexpr (PN && GRAD) {
        const Tab<T> &tb = TabSel<T>::get(P);
        for (int i = tid; i < 4 * P * P; i += nt) {
            const int w = i / (P * P), r = i - w * (P * P), tau = r / P, m = r - tau * P;
            rt[i] = w == 0 ? tb.prvL[tau][m] : (w == 1 ? tb.prdL[tau][m] : (w == 2 ? tb.prvR[tau][m] : tb.prdR[tau][m]));
        }
    }

    // ghost slots of non-periodic ends: mir = 1 mirrored ghost (odd normal
    // modes negated), 2 reflecting wall (the same, and the normal momentum
    // negated as a whole)
    for (int s = tid; s <= C; s += nt) {
        int ca = a0 + s - 1;
        int m = 0;
        if (geo.bc[AX] == 0) {
            if (ca < 0 || ca >= na) ca = ((ca % na) + na) % na;   // pencils may be longer than the axis
        } else {
            if (ca < 0) {
                ca = 0;
                m = geo.bc[AX];
            } else if (ca >= na) {
                ca = na - 1;
                m = geo.bc[AX];
            }
        }
        int cc[3] = {co[0], co[1], co[2]};
        cc[AX] = ca;
        cellidx[s] = cc[0] + (long long)geo.n[0] * (cc[1] + (long long)geo.n[1] * cc[2]);
        mir[s] = m;
    }
    __syncthreads();
    // normal contraction, one item per (slot s, field f, transverse mode t):
    // the p weights of the line along the normal are read from HBM (mirrored
    // ghost: odd normal modes negated); slot s is the lower cell of face s
    // (trace P~(+1) and the lower-side recovery partial sums) and the upper
    // cell of face s - 1 (trace P~(-1) and the upper-side partial sums).  The
    // two sides' partial sums are added after the barrier.
    {
        const Tab<T> &tb = TabSel<T>::get(P);
        T *A2u = Sx, *A3u = Sx + Q;                       // upper-side partial sums
        for (int q = tid; q < (C + 1) * F * K; q += nt) {
            const int sf = q / K;
            const int t = q - sf * K;
            const int sl = sf / F, f = sf - sl * F;
            const int lo = t % S, hi = t / S;
            const double *src = a.w + cellidx[sl] * FNP + f * NM + lo + hi * S * P;
            const int mk = mir[sl];
            const bool mr = mk != 0;                       // odd modes negated
            const bool wn = mk == 2 && f == 1 + AX;        // wall: normal momentum negated
            T x[P];
            // P_n: the line's recovery vectors belong to its transverse degree
            // tau (data of normal degree <= n - tau recovered to n + 1 - tau)
            int tau = 0;
            if constexpr (PN) {
                const int t0 = lo + hi * S * P;            // tensor index of normal digit 0
                tau = t0 % P + (t0 / P) % P + t0 / (P * P);
                const double *cp = a.w + cellidx[sl] * FNP + f * NM;
                if constexpr (AX == 0) {
                    // the x-line of transverse degrees (l_y, l_z) is stored contiguously
                    const double *lp = cp + BS::off(t0 / P % P, t0 / (P * P));
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const double v = m < P - tau ? lp[m] : 0.0;
                        x[m] = (T)(((mr && (m & 1)) != wn) ? -v : v);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const int ti = t0 + m * S;
                        const int id = BS::idx(ti % P, (ti / P) % P, ti / (P * P));
                        const double v = id >= 0 ? cp[id] : 0.0;
                        x[m] = (T)(((mr && (m & 1)) != wn) ? -v : v);
                    }
                }
            } else if (AX == 0 && P % 2 == 0) {
#pragma unroll
                for (int m = 0; m < P; m += 2) {
                    const DV<2> v = ldv<2>(src + m);
                    x[m] = (T)(wn ? -v.x[0] : v.x[0]);
                    x[m + 1] = (T)((mr != wn) ? -v.x[1] : v.x[1]);
                }
            } else {
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const double v = src[m * S];
                    x[m] = (T)(((mr && (m & 1)) != wn) ? -v : v);
                }
            }
            // table row of the recovery vectors (lines beyond the basis, tau > n,
            // hold zeros: any row gives their exact 0; the LDS table has p rows)
            const int trow = tau < P ? tau : P - 1;
            const int pt = ppos<P, PP>(t);
            if (sl < C) {
                const int qa = (sl * F + f) * NAF + pt;
                T tl = T(0);
#pragma unroll
                for (int m = 0; m < P; ++m) tl = fma(tb.ep[m], x[m], tl);
                A[0 * Q + qa] = tl;
                if (GRAD) {
                    const T *vL = PN ? rt + trow * P : tb.rvL, *dL = PN ? rt + (P + trow) * P : tb.rdL;
                    T rv = T(0), rn = T(0);
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        rv = fma(vL[m], x[m], rv);
                        rn = fma(dL[m], x[m], rn);
                    }
                    A[2 * Q + qa] = rv;
                    A[3 * Q + qa] = rn;
                }
            }
            if (sl > 0) {
                const int qa = ((sl - 1) * F + f) * NAF + pt;
                T tr = T(0);
#pragma unroll
                for (int m = 0; m < P; ++m) tr = fma(tb.em[m], x[m], tr);
                A[1 * Q + qa] = tr;
                if (GRAD) {
                    const T *vR = PN ? rt + (2 * P + trow) * P : tb.rvR, *dR = PN ? rt + (3 * P + trow) * P : tb.rdR;
                    T rv = T(0), rn = T(0);
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        rv = fma(vR[m], x[m], rv);
                        rn = fma(dR[m], x[m], rn);
                    }
                    A2u[qa] = rv;
                    A3u[qa] = rn;
                }
            }
        }
        __syncthreads();
        if (GRAD) {
            for (int i = tid; i < Q; i += nt) {
                A[2 * Q + i] += A2u[i];
                A[3 * Q + i] += A3u[i];
            }
            __syncthreads();
        }
    }

    // transverse transforms to the face Gauss points
    const T *tLp, *tRp, *utp = nullptr, *rnp = nullptr, *d1p = nullptr, *d2p = nullptr;
    if (D == 2) {
        line_pass_pad<P, 1, 0, T, M_B, false, NTC, PP>(A, Sx, NA * C * F);
        if (GRAD) line_pass_pad<P, 1, 0, T, M_BD, false, NTC, PP>(A + 2 * Q, Sx + 4 * Q, C * F);
        __syncthreads();
        tLp = Sx;
        tRp = Sx + Q;
        utp = Sx + 2 * Q;
        rnp = Sx + 3 * Q;
        d1p = Sx + 4 * Q;
    } else {
        // (t1, t2) = transverse axes of the face in ascending order
        line_pass_pad<P, 2, 0, T, M_B, false, NTC, PP>(A, Sx, NA * C * F);
        if (GRAD) line_pass_pad<P, 2, 0, T, M_BD, false, NTC, PP>(A + 2 * Q, Sx + 4 * Q, C * F);
        __syncthreads();
        line_pass_pad<P, 2, 1, T, M_B, false, NTC, PP>(Sx, A, NA * C * F);
        __syncthreads();
        if (GRAD) {
            line_pass_pad<P, 2, 1, T, M_BD, false, NTC, PP>(Sx + 2 * Q, Sx, C * F);
            line_pass_pad<P, 2, 1, T, M_B, false, NTC, PP>(Sx + 4 * Q, Sx + Q, C * F);
            __syncthreads();
        }
        tLp = A;
        tRp = A + Q;
        utp = A + 2 * Q;
        rnp = A + 3 * Q;
        d2p = Sx;
        d1p = Sx + Q;
    }

    // point fluxes: F = HLLC(u-, u+) - vis, vis = F_NS(u~, grad u~) + eps grad u~
    //   (viscous / AV part from the recovered state, Sec. 3.2 and 4.1)
    const T gamma = (T)ph.gamma;
    const Tab<T> &tb = TabSel<T>::get(P);
    T *fb = (T *)a.fb + geo.fb_off[AX];
    auto viscous = [&](int c, int kp, T *vis) {
        T ut[MAXF];
        T g[D][MAXF];
        constexpr int T1 = (AX == 0) ? 1 : 0;             // transverse axes, ascending
        constexpr int T2 = (D == 3) ? ((AX == 2) ? 1 : 2) : 0;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const int idx = (c * F + f) * NAF + kp;
            ut[f] = utp[idx];
            g[AX][f] = rnp[idx] * (T)ph.inv_fh;
            g[T1][f] = d1p[idx] * (T)ph.two_over_h;
            if (D == 3) g[T2][f] = d2p[idx] * (T)ph.two_over_h;
        }
        const Prim<D, T> s = primitives<D, T>(ut, gamma);
#pragma unroll
        for (int f = 0; f < Fc; ++f) vis[f] = T(0);
        if (Fld<D, PH>::NS || ph.ns_on) {
            T fv[D + 2];
            const NsGrad<D, T> ng = ns_grad<D, T>(ut, s, g);
            ns_flux<D, T>(s, ng, AX, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
            for (int f = 0; f < D + 2; ++f) vis[f] = fv[f];
            // tracer diffusion eta rho d_a c = eta (d_a(c rho) - c d_a rho)
            if (Fld<D, PH>::TR) vis[D + 2] = (T)ph.eta * (g[AX][D + 2] - ut[D + 2] * s.ir * g[AX][0]);
        }
        if (Fld<D, PH>::AV) {
            const T cs = sqrt(gamma * s.p * s.ir);
            const T eps = (T)ph.av_scale * clamp_alpha(ut[Fc], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
#pragma unroll
            for (int f = 0; f < Fc; ++f) vis[f] += eps * g[AX][f];
        }
    };
    auto riemann = [&](int c, int kp, T *Fh) {
        T uL[Fc], uR[Fc];
#pragma unroll
        for (int f = 0; f < Fc; ++f) {
            uL[f] = tLp[(c * F + f) * NAF + kp];
            uR[f] = tRp[(c * F + f) * NAF + kp];
        }
        hllc<D, T, Fc>(uL, uR, AX, gamma, Fh);
    };
    auto store = [&](int c, int k, const T *Fh) {
        T gk = tb.g[k % P];
        if (D == 3) gk *= tb.g[k / P];
        int cf[3] = {co[0], co[1], co[2]};
        cf[AX] = a0 + c;
        const long long nd0 = (AX == 0) ? nfa : geo.n[0];
        const long long nd1 = (AX == 1) ? nfa : geo.n[1];
        const long long fi = cf[0] + nd0 * (cf[1] + nd1 * cf[2]);
        T *dst = fb + fi * (long long)(Fc * K) + k;
#pragma unroll
        for (int f = 0; f < Fc; ++f) dst[f * K] = gk * Fh[f];
    };
    for (int q = tid; q < C * K; q += nt) {
        const int c = q / K, k = q - c * K;
        if (c >= nface) continue;
        const int kp = ppos<P, PP>(k);
        T Fh[Fc];
        riemann(c, kp, Fh);
        if (GRAD) {
            T vis[Fc];
            viscous(c, kp, vis);
#pragma unroll
            for (int f = 0; f < Fc; ++f) Fh[f] -= vis[f];
        }
        store(c, k, Fh);
    }
}

// Number of pencils of direction ax (ceil(nf/C) per line times the lines).
__device__ __forceinline__ long long pencils(const Geo &geo, int ax, int C)
{
    long long npen = (geo.nf[ax] + C - 1) / C;
    for (int b = 0; b < 3; ++b)
        if (b != ax) npen *= geo.n[b];
    return npen;
}

// Pencil pen of direction ax in line order (lines of the transverse cell
// coordinates, first transverse axis fastest; pencils along a line fastest),
// the enumeration of the grouped launches.  32-bit arithmetic (the host
// bounds the counts by 2^31).
__device__ __forceinline__ void pencil_coords(const Geo &geo, int C, int ax, long long pen, int *co, int &a0)
{
    const unsigned npl = (unsigned)((geo.nf[ax] + C - 1) / C);
    const unsigned line = (unsigned)pen / npl;
    a0 = (int)((unsigned)pen - line * npl) * C;
    co[0] = co[1] = co[2] = 0;
    unsigned r = line;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if (b != ax) {
            const unsigned nb = (unsigned)geo.n[b];
            const unsigned q = r / nb;
            co[b] = (int)(r - q * nb);
            r = q;
        }
}

// Block -> pencil map of the single-box face launch (grid of face_grid):
// bricks of C cells per axis, x fastest; each brick's pencils of all
// directions (C^(D-1) per direction, the directions alternating) are
// consecutive blocks, so the three reads of a cell (one per direction) fall
// close together in time on one XCD and the second and third come from L2.
// Returns false for the blocks of a brick beyond the mesh.
__device__ __forceinline__ bool face_brick(const Geo &geo, int D, int C, int &ax, int *co, int &a0)
{
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    const unsigned L = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
    const unsigned K1 = (D == 3) ? (unsigned)(C * C) : (unsigned)C;   // pencils per direction and brick
    const unsigned S = (unsigned)D * K1;
    const unsigned brick = L / S, s = L - brick * S;
    ax = (int)(s % (unsigned)D);
    const unsigned j = s / (unsigned)D;
    const unsigned B0 = (unsigned)((geo.nf[0] + C - 1) / C), B1 = (unsigned)((geo.nf[1] + C - 1) / C);
    const unsigned r = brick / B0;
    const unsigned b[3] = {brick - r * B0, r % B1, r / B1};
    const int t1 = (ax == 0) ? 1 : 0, t2 = (ax == 2) ? 1 : 2;   // transverse axes
    a0 = (int)(b[ax] * (unsigned)C);
    if (a0 >= geo.nf[ax]) return false;
    co[0] = co[1] = co[2] = 0;
    co[t1] = (int)(b[t1] * (unsigned)C + j % (unsigned)C);
    if (co[t1] >= geo.n[t1]) return false;
    if (D == 3) {
        co[t2] = (int)(b[t2] * (unsigned)C + j / (unsigned)C);
        if (co[t2] >= geo.n[t2]) return false;
    }
    return true;
}

template <int D, int P, typename T, int PH, int CC = 0, int NTC = 0>
__device__ __forceinline__ void face_dispatch(const Phys &ph, const Geo &geo, const FaceArgs &a, unsigned char *smem,
                                              int ax, const int *co, int a0)
{
    if (ax == 0)
        face_body<D, P, 0, T, PH, CC, NTC>(ph, geo, a, smem, co, a0);
    else if (ax == 1)
        face_body<D, P, 1, T, PH, CC, NTC>(ph, geo, a, smem, co, a0);
    else if (D == 3)
        face_body<D, P, (D == 3 ? 2 : 0), T, PH, CC, NTC>(ph, geo, a, smem, co, a0);
}

// The CFL finalize carried by a face launch: block (0, 0) reduces the CFL
// kernel's per-block (c_s, |v|) maxima (wave shuffles, then 16 doubles of
// LDS across the waves) and writes dt = f_CFL h / (2 p (c_max + v_max)).
// The next kernel on the stream (the volume kernel of the same stage) reads it.
__device__ __forceinline__ void face_cfl_finalize(const FaceArgs &a, unsigned char *smem)
{
    if (!a.cfl_part || blockIdx.x != 0 || blockIdx.y != 0 || blockIdx.z != 0) return;
    const int nt = blockDim.x;
    const double2 *pp = (const double2 *)a.cfl_part;
    double c = 0.0, v = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < a.cfl_nblk; b += nt) {
        const double2 x = pp[b];
        c = nanmax(c, x.x);
        v = nanmax(v, x.y);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c = nanmax(c, __shfl_xor(c, off));
        v = nanmax(v, __shfl_xor(v, off));
    }
    double *red = (double *)smem;
    if ((threadIdx.x & 63) == 0) {
        red[2 * (threadIdx.x >> 6)] = c;
        red[2 * (threadIdx.x >> 6) + 1] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nt / 64; ++w) {
            c = nanmax(c, red[2 * w]);
            v = nanmax(v, red[2 * w + 1]);
        }
        const double dt = a.cfl_num / (c + v);
        a.cfl_res[0] = dt;
        a.cfl_res[1] = c;
        a.cfl_res[2] = v;
        if (a.cfl_dt_copy) a.cfl_dt_copy[0] = dt;
    }
    __syncthreads();   // the face work reuses the LDS
}

template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) face_kernel(Phys ph, Geo geo, FaceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    face_cfl_finalize(a, smem);
    int ax, co[3], a0;
    if (!face_brick(geo, D, a.faces_per_block, ax, co, a0)) return;
    face_dispatch<D, P, T, PH>(ph, geo, a, smem, ax, co, a0);
}

// Face kernel with the pencil length C and block size NT fixed at compile
// time; instantiated for the tuned tiles and launched only with
// blockDim.x == NT and faces_per_block == C.
template <int D, int P, typename T, int PH, int C, int NT>
__global__ void __launch_bounds__(NT) face_kernel_fixed(Phys ph, Geo geo, FaceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.faces_per_block != C) return;   // host selection error
    face_cfl_finalize(a, smem);
    int ax, co[3], a0;
    if (!face_brick(geo, D, C, ax, co, a0)) return;
    face_dispatch<D, P, T, PH, C, NT>(ph, geo, a, smem, ax, co, a0);
}

// Index of the box owning flat block b of a grouped launch.
__device__ __forceinline__ int owner_box(const BoxDesc *boxes, int nbox, long long b, int which)
{
    // largest i with start[i] <= b (starts are non-decreasing, start[0] = 0):
    // binary search, about log2(nbox) uniform loads
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxes[mid].start[which] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Grouped face kernel: every box of one (dim, order) group; flat block index
// -> (box, direction, pencil).
template <int D, int P, typename T, int PH, int CC, int NTC>
__device__ __forceinline__ void face_batched_body(const BoxDesc *boxes, int nbox, int stage_cur)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = xcd_block(blockIdx.x, gridDim.x);
    const int i = owner_box(boxes, nbox, b, 1);
    const Phys &ph = boxes[i].ph;
    const Geo &geo = boxes[i].geo;
    FaceArgs a;
    a.w = boxes[i].reg[stage_cur];
    a.fb = boxes[i].fb;
    a.faces_per_block = boxes[i].faces_per_block;
    a.cfl_part = nullptr;
    if (CC > 0 && a.faces_per_block != CC) return;   // host selection error
    long long loc = b - boxes[i].start[1];
    for (int ax = 0; ax < D; ++ax) {
        const long long n = pencils(geo, ax, a.faces_per_block);
        if (loc < n) {
            int co[3], a0;
            pencil_coords(geo, a.faces_per_block, ax, loc, co, a0);
            face_dispatch<D, P, T, PH, CC, NTC>(ph, geo, a, smem, ax, co, a0);
            return;
        }
        loc -= n;
    }
}

template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) face_kernel_batched(const BoxDesc *boxes, int nbox, int stage_cur)
{
    face_batched_body<D, P, T, PH, 0, 0>(boxes, nbox, stage_cur);
}

// Grouped face kernel with the pencil length C and block size NT fixed.
template <int D, int P, typename T, int PH, int C, int NT>
__global__ void __launch_bounds__(NT) face_kernel_batched_fixed(const BoxDesc *boxes, int nbox, int stage_cur)
{
    face_batched_body<D, P, T, PH, C, NT>(boxes, nbox, stage_cur);
}


// LDS bytes of the face kernel for pencils of C faces: slot indices, a
// scratch of 5 C F p^(d-1) and the contraction results A (NA C F p^(d-1)).
template <int D, int P, typename T, int PH>
size_t face_lds_bytes(int C)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    constexpr int F = Fld<D, PH>::F;
    constexpr int PP = FacePad<P>::PP;
    const size_t hdr = (((C + 1) * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16;
    const size_t Q = (size_t)C * F * (PP * K / P);
    const size_t NA = Fld<D, PH>::GRAD ? 4 : 2;
    const size_t rt = (Fld<D, PH>::PN && Fld<D, PH>::GRAD) ? 4 * P * P : 0;   // P_n recovery vectors
    const size_t tot = 5 * Q + NA * Q + rt;
    return hdr + sizeof(T) * tot;
}

// Sensor top modes (Sec. 4.1: absent at the next lower order) by storage
// index: max_a l_a = n for Q_n, total degree n for P_n.
template <int D, int P, bool PN>
__device__ __forceinline__ bool is_top(int m)
{
    if constexpr (PN) {
        // walk the P_n storage order to the degrees of m
        int lz = 0, ly = 0;
        while (true) {
            const int nl = Basis<D, P, true>::len(ly, lz);
            if (m < nl) return m + ly + lz == P - 1;
            m -= nl;
            if (++ly > P - 1 - lz) {
                ly = 0;
                ++lz;
            }
        }
    } else {
        bool tp = false;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            tp = tp || (m % P == P - 1);
            m /= P;
        }
        return tp;
    }
}

// ---------------------------------------------------------------------------
// volume kernel
// ---------------------------------------------------------------------------

// LDS header of the volume kernel: face indices [C][D][2] (long long), wiggle
// source [C] and new cell means [C][D+2] (double), the block's error flag;
// rounded to 16 bytes.  Then the FP64 surface sums of the cell means
// [D+2][C][p^(d-1)] (double): per lift line, the sum over the axes of the
// lower minus the upper face flux at its face point.
template <int D>
__host__ __device__ constexpr size_t vol_hdr_bytes(int C)
{
    return ((C * (2 * D * sizeof(long long) + (1 + D + 2) * sizeof(double)) + sizeof(int) + 15) / 16) * 16;
}

template <int D, int P>
__host__ __device__ constexpr size_t vol_m0_bytes(int C, int Fc)
{
    return (size_t)Fc * C * ipow(P, D - 1) * sizeof(double);
}

// CC, NTC, FO: cells per block, threads per block and forcing (0 off, 1 on)
// fixed at compile time (0 / 0 / -1 = taken from the launch).  Fixing them
// removes the runtime tile arithmetic; the results are the same bits.
template <int D, int P, typename T, int PH, int CC = 0, int NTC = 0, int FO = -1>
__device__ __forceinline__ void vol_body(const Phys &ph, const Geo &geo, const VolArgs &a, unsigned char *smem,
                                         long long tile)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    constexpr int Fc = Fld<D, PH>::Fc;
    constexpr int F = Fld<D, PH>::F;
    constexpr bool GRAD = Fld<D, PH>::GRAD;
    constexpr bool PN = Fld<D, PH>::PN;
    using BS = Basis<D, P, PN>;
    constexpr int NM = BS::NM;                // stored modes per field
    constexpr int FNP = F * NM;               // stored weights per cell
    const bool forced = FO >= 0 ? FO == 1 : a.forcing != nullptr;
    const int C = CC > 0 ? CC : a.cells_per_block;
    constexpr int NAP = Pad<P>::PP * NP / P;  // padded per-cell array
    const int CNP = C * NAP;                  // one field of the tile
    const int tid = threadIdx.x, nt = NTC > 0 ? NTC : (int)blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = tile * C;

    // LDS, field-major: Ub [field][cell][point] (point values, then sources),
    // G [axis][field][cell][point] (gradients, then fluxes); points in the
    // padded layout of Pad<P>.  The ping-pong buffer of the contraction
    // passes lives in G's space (D F >= F arrays), which is free outside
    // the gradient / flux phases.  The driving field is read at the Gauss
    // points from HBM by the source step (no LDS).
    long long *fidx = (long long *)smem;      // [C][D][2] lower/upper face index per axis
    double *cellv = (double *)(fidx + 2 * D * C);   // [C]: wiggle source
    double *cmean = cellv + C;                // [C][D+2]: new cell means (checks)
    int *blkflag = (int *)(cmean + C * (D + 2));
    double *m0s = (double *)(smem + vol_hdr_bytes<D>(C));   // [Fc][C][K] FP64 surface sums
    T *Ub = (T *)(smem + vol_hdr_bytes<D>(C) + vol_m0_bytes<D, P>(C, Fc));
    T *G = Ub + F * CNP;
    T *X0 = (D == 3) ? G : Ub;     // the last of the D passes lands in Ub
    T *X1 = (D == 3) ? Ub : G;
    const Tab<T> &tb = TabSel<T>::get(P);

    // 1. per-cell data (the weights themselves are read by the first pass)
    if (tid == 0) *blkflag = 0;
    for (int cl = tid; cl < C; cl += nt) {
        long long cc = c0 + cl;
        if (cc >= NC) cc = NC - 1;
        // coordinates and face indices in 32 bits (the host bounds them by 2^31)
        const unsigned u = (unsigned)cc, n0 = (unsigned)geo.n[0], n1 = (unsigned)geo.n[1];
        const unsigned r0 = u / n0;
        const unsigned co[3] = {u - r0 * n0, r0 % n1, r0 / n1};
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const unsigned nfa = (unsigned)geo.nf[ax];
            unsigned flo = 0, fhi = 0, mul = 1;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const unsigned nb = (b == ax) ? nfa : (unsigned)geo.n[b];
                unsigned ilo = co[b], ihi = co[b];
                if (b == ax) {
                    ihi = co[b] + 1;
                    if (ihi >= nfa) ihi -= nfa;   // periodic wrap (outflow has nf = n + 1)
                }
                flo += ilo * mul;
                fhi += ihi * mul;
                mul *= nb;
            }
            fidx[(cl * D + ax) * 2] = flo;
            fidx[(cl * D + ax) * 2 + 1] = fhi;
        }
        if (Fld<D, PH>::AV) {
            // sensor S of the current state and the wiggle source (Sec. 4.1)
            const double *wr = a.cur + cc * FNP;
            double all = 0.0, top = 0.0;
            for (int m = 0; m < NM; ++m) {
                const double x = wr[m];
                all += x * x;
                if (is_top<D, P, PN>(m)) top += x * x;
            }
            const double Sv = all > 0.0 ? top / all : 0.0;
            const double Rp = a.R_prev ? a.R_prev[cc] : 0.0;
            cellv[cl] = (Sv > ph.s_thr) ? ph.f_w * fmax(0.0, Rp) : 0.0;
        }
    }
    __syncthreads();

    // 2. point values of all fields: one operator pass per axis.  The pass
    //    along x reads each line's p modal weights (contiguous in HBM)
    //    straight from the state, so the weights never pass through LDS;
    //    the same FMA chain as the LDS passes.
    // With a fixed tile, line q = tid + r NT of this pass (r < KEEP) is also
    // line r of the final projection / RK pass of this thread: its FP64
    // weights are kept in registers for the RK combination (no second read).
    // (2D only: in 3D the kept registers pushed the forced kernel into SGPR
    // spills and were measured slower)
    constexpr int KEEP0 = (CC > 0 && NTC > 0 && D == 2) ? (CC * F * K + NTC - 1) / NTC : 0;
    constexpr int KEEP = (KEEP0 * P <= 8) ? KEEP0 : 0;
    double pcu[KEEP > 0 ? KEEP : 1][P];
    {
        constexpr int VWL = (P % 2 == 0) ? 2 : 1;       // state weights per load
        const int nitems = F * C * K;                   // K = p^(d-1) lines per array
        auto first_line = [&](int q, double *keep) {
            const int arr = q / K, t = q - arr * K;
            const int f = arr / C, c = arr - f * C;
            long long cc = c0 + c;
            if (cc >= NC) cc = NC - 1;                  // tail cells: copies of the last cell
            T x[P];
            if constexpr (PN) {
                // the line's l_x modes (zeros above total degree n)
                const int ly = t % P, lz = t / P;
                const int o0 = BS::off(ly, lz), nl = BS::len(ly, lz);
                const double *src = a.cur + cc * FNP + f * NM + o0;
#pragma unroll
                for (int k = 0; k < P; ++k) x[k] = (T)(k < nl ? src[k] : 0.0);
            } else {
                const double *src = a.cur + cc * FNP + f * NP + t * P;
#pragma unroll
                for (int k = 0; k < P; k += VWL) {
                    const DV<VWL> v = ldv<VWL>(src + k);
#pragma unroll
                    for (int h = 0; h < VWL; ++h) {
                        x[k + h] = (T)v.x[h];
                        if (keep) keep[k + h] = v.x[h];
                    }
                }
            }
            const int o = pad_line_offset<P, D, 0>(q);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                T acc = T(0);
#pragma unroll
                for (int k = 0; k < P; ++k) acc = fma(mat<P, T, M_B>(k, i), x[k], acc);
                X1[o + i] = acc;
            }
        };
#pragma unroll
        for (int r = 0; r < KEEP; ++r)
            if (tid + r * nt < nitems) first_line(tid + r * nt, pcu[r]);
        for (int q = tid + KEEP * nt; q < nitems; q += nt) first_line(q, nullptr);
    }
    __syncthreads();
    line_pass_pad<P, D, 1, T, M_B, false, NTC>(X1, X0, F * C);
    __syncthreads();
    if (D == 3) {
        line_pass_pad<P, D, (D == 3 ? 2 : 0), T, M_B, false, NTC>(X0, X1, F * C);
        __syncthreads();
    }
    T *U = (D == 3) ? X1 : X0;
    T *Wk = (D == 3) ? X0 : X1;

    // 3. collocation gradients d/dxi of the stored fields
    if (GRAD) {
        line_pass_pad<P, D, 0, T, M_D, false, NTC>(U, G, F * C);
        line_pass_pad<P, D, 1, T, M_D, false, NTC>(U, G + F * CNP, F * C);
        if (D == 3) line_pass_pad<P, D, (D == 3 ? 2 : 0), T, M_D, false, NTC>(U, G + 2 * F * CNP, F * C);
        __syncthreads();
    }

    // 4. point fluxes (weighted by the volume Gauss weights) and sources
    const T gamma = (T)ph.gamma;
    for (int qq = tid; qq < C * NP; qq += nt) {
        const int cq = qq / NP, j = qq - cq * NP;
        const int q = cq * NAP + ppos<P>(j);   // padded position of point j of cell cq
        T u[F + D];
        if (forced) {
            // driving field at this Gauss point (tail cells: the last cell's)
            long long cc = c0 + cq;
            if (cc >= NC) cc = NC - 1;
            const T *sp = (const T *)a.forcing + cc * (D * NP) + j;
#pragma unroll
            for (int i = 0; i < D; ++i) u[F + i] = sp[i * NP];
        }
#pragma unroll
        for (int f = 0; f < F; ++f) u[f] = U[f * CNP + q];
        int jr = j;
        T wq = T(1);
#pragma unroll
        for (int b = 0; b < D; ++b) {
            wq *= tb.g[jr % P];
            jr /= P;
        }
        const Prim<D, T> s = primitives<D, T>(u, gamma);
        T g[D][MAXF];
        if (GRAD) {
#pragma unroll
            for (int b = 0; b < D; ++b)
#pragma unroll
                for (int f = 0; f < F; ++f) g[b][f] = G[(b * F + f) * CNP + q] * (T)ph.two_over_h;
        }
        T eps = T(0), cs = T(0);
        if (Fld<D, PH>::AV) {
            cs = sqrt(gamma * s.p * s.ir);
            eps = (T)ph.av_scale * clamp_alpha(u[Fc], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
        }
        NsGrad<D, T> ng;
        if (GRAD) ng = ns_grad<D, T>(u, s, g);
#pragma unroll
        for (int b = 0; b < D; ++b) {
            T fl[Fc];
            euler_flux<D, T>(u, s, b, fl);
            if (Fld<D, PH>::TR) fl[D + 2] = u[D + 2] * s.v[b];
            if (Fld<D, PH>::NS || (Fld<D, PH>::AV && ph.ns_on)) {
                T fv[D + 2];
                ns_flux<D, T>(s, ng, b, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
                for (int f = 0; f < D + 2; ++f) fl[f] -= fv[f];
                if (Fld<D, PH>::TR) fl[D + 2] -= (T)ph.eta * (g[b][D + 2] - u[D + 2] * s.ir * g[b][0]);
            }
            if (Fld<D, PH>::AV) {
#pragma unroll
                for (int f = 0; f < Fc; ++f) fl[f] -= eps * g[b][f];
            }
#pragma unroll
            for (int f = 0; f < Fc; ++f) G[(b * F + f) * CNP + q] = wq * fl[f];
        }
        // sources, scaled to the common prefactor: Q = (h/2) w_j src
        const T hw = (T)ph.half_h * wq;
        T src[Fc];
#pragma unroll
        for (int f = 0; f < Fc; ++f) src[f] = T(0);
        if (forced) {
            T sv = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                src[1 + i] = s.rho * u[F + i];
                sv += u[F + i] * u[1 + i];
            }
            src[D + 1] = sv;
        }
#pragma unroll
        for (int f = 0; f < Fc; ++f) U[f * CNP + q] = hw * src[f];
        if (Fld<D, PH>::AV) {
            const T asrc = (T)ph.f_v * fmax(T(0), -ng.div) + (T)cellv[cq] - u[Fc] * cs * (T)ph.sink;
            U[Fc * CNP + q] = hw * asrc;
        }
    }
    __syncthreads();

    // Global reads of the later phases are issued early, after the flux
    // phase (the register peak), so their latency overlaps the D^T, lift and
    // projection passes: the face fluxes of the lift and the RK inputs of the
    // first NLD groups of each thread (the rest, if any, are read where they
    // are used).  With a fixed tile the counts are exact, and the lift is
    // fused into the D^T passes: line q of the D^T pass along a is the line
    // (field f, cell c, transverse point t) whose end points the two a-faces
    // of cell c at face point t lift.
    constexpr bool FUSED = CC > 0 && NTC > 0;
    constexpr int NLF = 1;                                         // lift rounds read early (generic tile)
    constexpr int NDT = FUSED ? (CC * Fc * K + NTC - 1) / NTC : 1;   // D^T lines per thread
    // lines of the final (x) projection pass per thread, and how many of them
    // get their RK inputs read early (p doubles per array per line)
    constexpr int NBL = KEEP;                      // their cur weights are already in pcu
    const int nlift = C * Fc * K;
    auto lift_load = [&](int q, T *Fl, T *Fu) {
        const bool act = q < nlift;
        const int c = act ? q / (Fc * K) : 0;
        const int r = q - c * (Fc * K);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const T *fb = (const T *)a.fb + geo.fb_off[ax];
            const long long flo = fidx[(c * D + ax) * 2], fhi = fidx[(c * D + ax) * 2 + 1];
            Fl[ax] = act ? fb[flo * (Fc * K) + r] : T(0);
            Fu[ax] = act ? fb[fhi * (Fc * K) + r] : T(0);
        }
    };
    T lfl[NLF][D], lfu[NLF][D];
    T dlf[D][NDT][2];
    if constexpr (FUSED) {
#pragma unroll
        for (int r = 0; r < NDT; ++r) {
            const int q = tid + r * nt;
            const bool act = q < nlift;
            const int arr = act ? q / K : 0;            // array (f, c) of the U layout: f C + c
            const int f = arr / C, c = arr - f * C;
            const int t = q - arr * K;                  // transverse point = face point
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                const T *fb = (const T *)a.fb + geo.fb_off[ax];
                const long long flo = fidx[(c * D + ax) * 2], fhi = fidx[(c * D + ax) * 2 + 1];
                dlf[ax][r][0] = act ? fb[flo * (Fc * K) + f * K + t] : T(0);
                dlf[ax][r][1] = act ? fb[fhi * (Fc * K) + f * K + t] : T(0);
            }
            // FP64 surface sum of this line's face point (the mode-0 RHS of
            // a conserved field is the sum of these over the face points)
            if (act) {
                double sm = 0.0;
#pragma unroll
                for (int ax = 0; ax < D; ++ax) sm += (double)dlf[ax][r][0] - (double)dlf[ax][r][1];
                m0s[q] = sm;
            }
        }
    } else {
#pragma unroll
        for (int rr = 0; rr < NLF; ++rr) lift_load(tid + rr * nt, lfl[rr], lfu[rr]);
        // FP64 surface sums per lift line (f, c, face point), same order as above
        for (int q = tid; q < nlift; q += nt) {
            T Fl[D], Fu[D];
            lift_load(q, Fl, Fu);
            const int c = q / (Fc * K);
            const int r = q - c * (Fc * K);
            const int f = r / K, k = r - f * K;
            double sm = 0.0;
#pragma unroll
            for (int ax = 0; ax < D; ++ax) sm += (double)Fl[ax] - (double)Fu[ax];
            m0s[(f * C + c) * K + k] = sm;
        }
    }

    const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
    constexpr int VWL = (P % 2 == 0) ? 2 : 1;      // weights per access along a line
    const int nx = F * C * K;                      // lines of the final projection pass
    // RK inputs of a final-pass line: p consecutive weights of cur / base / x2
    auto rk_load = [&](int q, double *cu, double *ba, double *x2, bool with_cur) {
        const int arr = q / K, t = q - arr * K;
        const int f = arr / C, c = arr - f * C;
        const long long cc = c0 + c;
        const bool ok = q < nx && cc < NC;
        if constexpr (PN) {
            const int ly = t % P, lz = t / P;
            const long long gi = cc * FNP + f * NM + BS::off(ly, lz);
            const int nl = BS::len(ly, lz);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const bool in = ok && k < nl;
                if (with_cur) cu[k] = in ? a.cur[gi + k] : 0.0;
                ba[k] = (in && a.base) ? a.base[gi + k] : 0.0;
                x2[k] = (in && a.x2) ? a.x2[gi + k] : 0.0;
            }
            return;
        }
        const long long gi = cc * FNP + f * NP + t * P;
#pragma unroll
        for (int k = 0; k < P; k += VWL) {
            const DV<VWL> zc = zdv<VWL>();
            const DV<VWL> vc = (ok && with_cur) ? ldv<VWL>(a.cur + gi + k) : zc;
            const DV<VWL> vb = (ok && a.base) ? ldv<VWL>(a.base + gi + k) : zc;
            const DV<VWL> vx = (ok && a.x2) ? ldv<VWL>(a.x2 + gi + k) : zc;
#pragma unroll
            for (int h = 0; h < VWL; ++h) {
                if (with_cur) cu[k + h] = vc.x[h];
                ba[k + h] = vb.x[h];
                x2[k + h] = vx.x[h];
            }
        }
    };
    double pba[NBL > 0 ? NBL : 1][P], px2[NBL > 0 ? NBL : 1][P];
#pragma unroll
    for (int r = 0; r < NBL; ++r) rk_load(tid + r * nt, pcu[r], pba[r], px2[r], false);

    // 5.-6. Q += sum_a [D_a^T (w f_a) + surface lift of the two a-faces], axis by axis
    if constexpr (FUSED) {
        dt_lift_pass<P, D, 0, T, NTC, NDT>(G, U, Fc * C * K, dlf[0]);
        __syncthreads();
        dt_lift_pass<P, D, 1, T, NTC, NDT>(G + F * CNP, U, Fc * C * K, dlf[1]);
        __syncthreads();
        if (D == 3) {
            dt_lift_pass<P, D, (D == 3 ? 2 : 0), T, NTC, NDT>(G + 2 * F * CNP, U, Fc * C * K, dlf[D - 1]);
            __syncthreads();
        }
    } else {
        // per axis: the D^T pass, then the lift of that axis, Q(i, k) +=
        // L_i(-1) F_lower(k) - L_i(+1) F_upper(k) (same summation order as
        // the fused passes, so both give the same bits)
        const int rounds = (nlift + nt - 1) / nt;          // uniform over the block
        auto lift_ax = [&](int ax, int q, T Fl, T Fu) {
            const bool act = q < nlift;
            const int c = act ? q / (Fc * K) : 0;
            const int r = q - c * (Fc * K);
            const int f = act ? r / K : 0, k = act ? r - f * K : 0;
            const int S = (ax == 0) ? 1 : (ax == 1 ? P : P * P);
            if (act) {
                const int lo = k % S, hi = k / S;
                T *po = U + f * CNP + c * NAP;
                const int j0 = lo + hi * S * P;
#pragma unroll
                for (int i = 0; i < P; ++i) po[ppos<P>(j0 + i * S)] += tb.Lm[i] * Fl - tb.Lp[i] * Fu;
            }
        };
        auto axis = [&](auto axc) {
            constexpr int AX = decltype(axc)::value;
            line_pass_pad<P, D, AX, T, M_DT, true, NTC>(G + AX * F * CNP, U, Fc * C);
            __syncthreads();
#pragma unroll
            for (int rr = 0; rr < NLF; ++rr)
                if (rr < rounds) lift_ax(AX, tid + rr * nt, lfl[rr][AX], lfu[rr][AX]);
            for (int rr = NLF; rr < rounds; ++rr) {
                T Fl[D], Fu[D];
                lift_load(tid + rr * nt, Fl, Fu);
                lift_ax(AX, tid + rr * nt, Fl[AX], Fu[AX]);
            }
            __syncthreads();
        };
        axis(std::integral_constant<int, 0>{});
        axis(std::integral_constant<int, 1>{});
        if constexpr (D == 3) axis(std::integral_constant<int, 2>{});
    }

    // 7.-8. point -> modal projection, last axis first; the pass along x
    //       (each line = p consecutive modal weights) is fused with the FP64
    //       RK combination and the write-back, p weights per thread.
    if (D == 3) {
        line_pass_pad<P, D, (D == 3 ? 2 : 0), T, M_BT, false, NTC>(U, Wk, F * C);
        __syncthreads();
        line_pass_pad<P, D, 1, T, M_BT, false, NTC>(Wk, U, F * C);
        __syncthreads();
    } else {
        line_pass_pad<P, D, 1, T, M_BT, false, NTC>(U, Wk, F * C);
        __syncthreads();
    }
    const T *Xs = (D == 3) ? U : Wk;   // input of the x pass
    T *Vl = (D == 3) ? Wk : U;         // the modal RHS, kept in LDS for the AV sensor rate
    const double pref = ph.pref;
    int bad = 0;
    auto xpass_rk = [&](int q, const double *cu, const double *ba, const double *x2) {
        const int arr = q / K, t = q - arr * K;
        const int f = arr / C, c = arr - f * C;
        const long long cc = c0 + c;
        const int o = pad_line_offset<P, D, 0>(q);
        T x[P], y[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = Xs[o + k];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < P; ++k) acc = fma(mat<P, T, M_BT>(k, i), x[k], acc);
            y[i] = acc;
        }
        // mode 0 of a conserved field without a volume source: the volume
        // term vanishes (Pt_0' = 0), so its RHS is the FP64 sum of the face
        // fluxes over the cell's faces (single-valued fluxes: the totals are
        // conserved to FP64 rounding also with an FP32 bulk)
        const bool m0 = t == 0 && f < Fc && (f == 0 || f == D + 2 || !forced);   // forcing: momentum, energy
        double y0 = (double)y[0];
        if (m0) {
            y0 = 0.0;
            for (int k = 0; k < K; ++k) y0 += m0s[arr * K + k];
            y[0] = (T)y0;
        }
        if (Fld<D, PH>::AV) {
#pragma unroll
            for (int i = 0; i < P; ++i) Vl[o + i] = y[i];
        }
        if (cc >= NC) return;
        // stored weights of this line: all p (Q_n), the first len (P_n)
        const int ly = t % P, lz = t / P;
        const int nl = BS::len(ly, lz);
        const long long gi = PN ? cc * FNP + f * NM + BS::off(ly, lz) : cc * FNP + f * NP + t * P;
        double ov[P], o2v[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const double L = pref * (i == 0 ? y0 : (double)y[i]);
            ov[i] = a.c_cur * cu[i] + a.c_L * dt * L;
            if (a.base) ov[i] += a.c_base * ba[i];
            o2v[i] = a.d_cur * cu[i] + a.d_L * dt * L + (a.x2 ? a.d_x2 * x2[i] : 0.0);
            if (!isfinite(ov[i]) && i < nl) bad |= 2;
        }
        if constexpr (PN) {
#pragma unroll
            for (int i = 0; i < P; ++i)
                if (i < nl) {
                    if (a.out2) a.out2[gi + i] = o2v[i];
                    a.out[gi + i] = ov[i];
                }
            if (t == 0 && f < D + 2) cmean[c * (D + 2) + f] = ov[0];
            return;
        }
#pragma unroll
        for (int k = 0; k < P; k += VWL) {
            DV<VWL> vo, vo2;
#pragma unroll
            for (int h = 0; h < VWL; ++h) {
                vo.x[h] = ov[k + h];
                vo2.x[h] = o2v[k + h];
            }
            if (a.out2) stv<VWL>(a.out2 + gi + k, vo2);
            stv<VWL>(a.out + gi + k, vo);
        }
        if (t == 0 && f < D + 2) cmean[c * (D + 2) + f] = ov[0];
    };
#pragma unroll
    for (int r = 0; r < NBL; ++r)
        if (tid + r * nt < nx) xpass_rk(tid + r * nt, pcu[r], pba[r], px2[r]);
    for (int q = tid + NBL * nt; q < nx; q += nt) {
        double cu[P], ba[P], x2[P];
        rk_load(q, cu, ba, x2, true);
        xpass_rk(q, cu, ba, x2);
    }
    if (bad) atomicOr(blkflag, bad);
    __syncthreads();

    // 9. per-cell checks (mean density and pressure) and, at stage 1, d ln S / dt
    for (int cl = tid; cl < C; cl += nt) {
        const long long cc = c0 + cl;
        if (cc >= NC) continue;
        const double *o = cmean + cl * (D + 2);
        const double rho = o[0];
        double m2 = 0.0;
        for (int i = 0; i < D; ++i) m2 += o[1 + i] * o[1 + i];
        const double pm = (ph.gamma - 1.0) * (o[D + 1] - 0.5 * m2 / rho);
        if (a.check && !(rho > 0.0 && pm > 0.0)) atomicOr(blkflag, 1);
        if constexpr (Fld<D, PH>::AV) if (a.R_out) {
            const double *wr = a.cur + cc * FNP;
            double Aa = 0.0, Tt = 0.0, ad = 0.0, td = 0.0;
            // density modes in tensor order j (P_n: those of the basis, read
            // from their storage index); Vl holds the modal RHS in the padded
            // tensor layout
            for (int m = 0; m < NP; ++m) {
                const int l0 = m % P, l1 = (m / P) % P, l2 = (D == 3) ? m / (P * P) : 0;
                const int id = BS::idx(l0, l1, l2);
                if (id < 0) continue;
                const double x = wr[id];
                const double xd = pref * (double)Vl[cl * NAP + ppos<P>(m)];
                Aa += x * x;
                ad += x * xd;
                const bool tp = PN ? (l0 + l1 + l2 == P - 1) : (l0 == P - 1 || l1 == P - 1 || (D == 3 && l2 == P - 1));
                if (tp) {
                    Tt += x * x;
                    td += x * xd;
                }
            }
            double R = 0.0;
            // rate kept only above the onset threshold (below it S is noise)
            if (Aa > 0.0 && Tt > 0.0 && Tt / Aa > ph.s_thr) {
                const double Sv = Tt / Aa;
                const double Sdot = 2.0 * (td * Aa - Tt * ad) / (Aa * Aa);
                R = Sdot / Sv;
            }
            a.R_out[cc] = R;
        }
    }
    __syncthreads();
    if (tid == 0 && *blkflag && a.flag) atomicOr(a.flag, *blkflag);
}

template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) vol_kernel(Phys ph, Geo geo, VolArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    vol_body<D, P, T, PH>(ph, geo, a, smem, xcd_block(blockIdx.x, gridDim.x));
}

// Volume kernel with the launch tile (C cells, NT threads) and the forcing
// switch fixed at compile time; instantiated for the tuned tiles.  The host
// launches it only with blockDim.x == NT, cells_per_block == C and forcing
// present iff FO == 1.
template <int D, int P, typename T, int PH, int C, int NT, int FO>
__global__ void __launch_bounds__(NT) vol_kernel_fixed(Phys ph, Geo geo, VolArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if ((FO == 1) != (a.forcing != nullptr) || a.cells_per_block != C) return;   // host selection error
    vol_body<D, P, T, PH, C, NT, FO>(ph, geo, a, smem, xcd_block(blockIdx.x, gridDim.x));
}

// Grouped volume/stage kernel over every box of one (dim, order) group.
// Body of the grouped volume kernel; CC / NTC as in vol_body (0 = from the
// launch).  Ensembles carry no forcing.
template <int D, int P, typename T, int PH, int CC, int NTC>
__device__ __forceinline__ void vol_batched_body(const BoxDesc *boxes, int nbox, const StageDesc &sd)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = xcd_block(blockIdx.x, gridDim.x);
    const int i = owner_box(boxes, nbox, b, 0);
    const BoxDesc &B = boxes[i];
    const Phys &ph = B.ph;
    const Geo &geo = B.geo;
    VolArgs a;
    a.cur = B.reg[sd.cur];
    a.base = sd.base >= 0 ? B.reg[sd.base] : nullptr;
    a.x2 = sd.x2 >= 0 ? B.reg[sd.x2] : nullptr;
    a.out = B.reg[sd.out];
    a.out2 = sd.out2 >= 0 ? B.reg[sd.out2] : nullptr;
    a.c_base = sd.c_base;
    a.c_cur = sd.c_cur;
    a.c_L = sd.c_L;
    a.d_x2 = sd.d_x2;
    a.d_cur = sd.d_cur;
    a.d_L = sd.d_L;
    a.dt_ptr = B.dt;
    a.dt = 0.0;
    a.fb = B.fb;
    a.forcing = nullptr;
    a.R_prev = nullptr;
    a.R_out = nullptr;
    a.flag = B.flag;
    a.check = 1;
    a.cells_per_block = B.cells_per_block;
    if (CC > 0 && B.cells_per_block != CC) return;   // host selection error
    vol_body<D, P, T, PH, CC, NTC, (CC > 0 ? 0 : -1)>(ph, geo, a, smem, b - B.start[0]);
}

template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) vol_kernel_batched(const BoxDesc *boxes, int nbox, StageDesc sd)
{
    vol_batched_body<D, P, T, PH, 0, 0>(boxes, nbox, sd);
}

// Grouped volume kernel with the tile fixed at compile time (every box of the
// group has cells_per_block == C; block size NT).
template <int D, int P, typename T, int PH, int C, int NT>
__global__ void __launch_bounds__(NT) vol_kernel_batched_fixed(const BoxDesc *boxes, int nbox, StageDesc sd)
{
    vol_batched_body<D, P, T, PH, C, NT>(boxes, nbox, sd);
}

// Gauss-point values of the driving-field coefficients (Sec. 7.1): arrays
// [cell][dim][modes] (FP64, in the layout of the basis) become point values
// [cell][dim][p^d] (j = j_x + p (j_y + p j_z)) in the bulk type T, by the line
// passes of the volume kernel's modal -> point transform (x, then y, then z;
// the same operator entries and FMA order, so the same bits).  The volume
// kernel reads them at its source step.  A block takes FA arrays.
template <int D, int P, typename T, bool PN>
__global__ void __launch_bounds__(256) forcing_points_kernel(const double *__restrict__ s, T *__restrict__ out,
                                                             long long narr)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    using BS = Basis<D, P, PN>;
    constexpr int NM = BS::NM;
    constexpr int FA = NP >= 256 ? 1 : 256 / NP;
    __shared__ T X[FA * NP], Y[FA * NP];
    const int tid = threadIdx.x, nt = blockDim.x;
    // grid-stride over groups of FA arrays (the grid is capped by the host)
    for (long long g0 = (long long)blockIdx.x * FA; g0 < narr; g0 += (long long)gridDim.x * FA) {
        for (int q = tid; q < FA * K; q += nt) {          // pass along x from the coefficients
            const int ar = q / K, t = q - ar * K;
            const long long g = g0 + ar;
            if (g >= narr) continue;
            const int ly = t % P, lz = t / P;
            const double *src = s + g * NM + (PN ? BS::off(ly, lz) : t * P);
            const int nl = PN ? BS::len(ly, lz) : P;
            T x[P];
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] = (T)(k < nl ? src[k] : 0.0);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                T acc = T(0);
#pragma unroll
                for (int k = 0; k < P; ++k) acc = fma(mat<P, T, M_B>(k, i), x[k], acc);
                X[ar * NP + t * P + i] = acc;
            }
        }
        __syncthreads();
        T *in = X, *o = Y;
#pragma unroll
        for (int ax = 1; ax < D; ++ax) {                  // passes along y (and z)
            const int S = ax == 1 ? P : P * P;
            for (int q = tid; q < FA * K; q += nt) {
                const int ar = q / K, t = q - ar * K;
                const int base = ar * NP + (ax == 1 ? (t % P) + P * P * (t / P) : t);
                T x[P];
#pragma unroll
                for (int k = 0; k < P; ++k) x[k] = in[base + k * S];
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    T acc = T(0);
#pragma unroll
                    for (int k = 0; k < P; ++k) acc = fma(mat<P, T, M_B>(k, i), x[k], acc);
                    o[base + i * S] = acc;
                }
            }
            __syncthreads();
            T *tmp = in;
            in = o;
            o = tmp;
        }
        for (int q = tid; q < FA * NP; q += nt) {
            const long long g = g0 + q / NP;
            if (g < narr) out[g * NP + q % NP] = in[q];
        }
        __syncthreads();   // X / Y are reused by the next group
    }
}

template <int D, int P, typename T, int PH>
size_t vol_lds_bytes(int C, int NU)
{
    constexpr int NP = Pad<P>::PP * ipow(P, D - 1);   // padded per-cell array
    constexpr int F = Fld<D, PH>::F;
    return vol_hdr_bytes<D>(C) + vol_m0_bytes<D, P>(C, Fld<D, PH>::Fc) +
           sizeof(T) * ((size_t)C * NU * NP + (size_t)C * D * F * NP);
}

// ---------------------------------------------------------------------------
// CFL kernel: maxima of c_s and |v| over the volume Gauss points (eq. timestep)
// ---------------------------------------------------------------------------


// Per-thread maxima of c_s and |v| over the Gauss points of one tile of C
// cells (accumulated into cmax / vmax; ends with a barrier, so the block can
// go on with another tile).
template <int D, int P, int PH>
__device__ __forceinline__ void cfl_tile(const Phys &ph, const Geo &geo, const CflArgs &a, unsigned char *smem,
                                         long long tile, double &cmax, double &vmax)
{
    constexpr int NP = ipow(P, D);
    constexpr int Fc = D + 2;
    constexpr bool PN = Fld<D, PH>::PN;
    using BS = Basis<D, P, PN>;
    constexpr int FNP = Fld<D, PH>::F * BS::NM;
    const int C = a.cells_per_block;
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = tile * C;
    constexpr int K = NP / P;
    constexpr int NAP = Pad<P>::PP * K;      // padded per-cell array
    const int CNP = C * NAP;
    // LDS field-major [field][cell][padded point]
    double *X0 = (double *)smem;
    double *X1 = X0 + Fc * CNP;
    // values at the Gauss points of the Fc conserved fields: the pass along x
    // reads each line's p modal weights straight from HBM, the others run in LDS
    {
        constexpr int VWL = (P % 2 == 0) ? 2 : 1;
        for (int q = tid; q < Fc * C * K; q += nt) {
            const int arr = q / K, t = q - arr * K;
            const int f = arr / C, c = arr - f * C;
            long long cc = c0 + c;
            if (cc >= NC) cc = NC - 1;
            double x[P];
            if constexpr (PN) {
                const int ly = t % P, lz = t / P;
                const double *src = a.w + cc * FNP + f * BS::NM + BS::off(ly, lz);
                const int nl = BS::len(ly, lz);
#pragma unroll
                for (int k = 0; k < P; ++k) x[k] = k < nl ? src[k] : 0.0;
            } else {
                const double *src = a.w + cc * FNP + f * NP + t * P;
#pragma unroll
                for (int k = 0; k < P; k += VWL) {
                    const DV<VWL> v = ldv<VWL>(src + k);
#pragma unroll
                    for (int h = 0; h < VWL; ++h) x[k + h] = v.x[h];
                }
            }
            const int o = pad_line_offset<P, D, 0>(q);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) acc = fma(mat<P, double, M_B>(k, i), x[k], acc);
                X1[o + i] = acc;
            }
        }
    }
    __syncthreads();
    line_pass_pad<P, D, 1, double, M_B, false>(X1, X0, Fc * C);
    __syncthreads();
    if (D == 3) {
        line_pass_pad<P, D, (D == 3 ? 2 : 0), double, M_B, false>(X0, X1, Fc * C);
        __syncthreads();
    }
    const double *U = (D == 3) ? X1 : X0;
    for (int q = tid; q < C * NP; q += nt) {
        const int c = q / NP, j = q - c * NP;
        if (c0 + c >= NC) continue;
        double u[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) u[f] = U[f * CNP + c * NAP + ppos<P>(j)];
        const Prim<D, double> s = primitives<D, double>(u, ph.gamma);
        double v2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) v2 += s.v[i] * s.v[i];
        cmax = nanmax(cmax, sqrt(ph.gamma * s.p * s.ir));   // NaN propagates into dt
        vmax = nanmax(vmax, sqrt(v2));
    }
    __syncthreads();
}

// Block maxima of the per-thread values into part[2 idx], part[2 idx + 1].
__device__ __forceinline__ void cfl_block_store(double *part, long long idx, double *red, double cmax, double vmax)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    red[tid] = cmax;
    red[nt + tid] = vmax;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[tid] = nanmax(red[tid], red[tid + s]);
            red[nt + tid] = nanmax(red[nt + tid], red[nt + tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[2 * idx] = red[0];
        part[2 * idx + 1] = red[nt];
    }
}

// LDS scratch of the block reduction, after the tile arrays.
template <int D, int P>
__device__ __forceinline__ double *cfl_red(unsigned char *smem, int C)
{
    return (double *)smem + 2 * (D + 2) * C * Pad<P>::PP * ipow(P, D - 1);
}

// Single-box CFL kernel: each block loops over the tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... and writes one partial, so the number of
// partials (the grid) stays bounded for any mesh.
template <int D, int P, int PH>
__global__ void __launch_bounds__(512) cfl_kernel(Phys ph, Geo geo, CflArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long ntiles = (geo.ncells + a.cells_per_block - 1) / a.cells_per_block;
    double cmax = 0.0, vmax = 0.0;
    for (long long t = blockIdx.x; t < ntiles; t += gridDim.x) cfl_tile<D, P, PH>(ph, geo, a, smem, t, cmax, vmax);
    cfl_block_store(a.part, blockIdx.x, cfl_red<D, P>(smem, a.cells_per_block), cmax, vmax);
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(512) cfl_kernel_batched(const BoxDesc *boxes, int nbox)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = blockIdx.x;
    const int i = owner_box(boxes, nbox, b, 2);
    const Phys &ph = boxes[i].ph;
    const Geo &geo = boxes[i].geo;
    CflArgs a;
    a.w = boxes[i].reg[0];
    a.part = boxes[i].cfl_part;
    a.cells_per_block = boxes[i].cfl_cells;
    double cmax = 0.0, vmax = 0.0;
    cfl_tile<D, P, PH>(ph, geo, a, smem, b - boxes[i].start[2], cmax, vmax);
    cfl_block_store(a.part, b - boxes[i].start[2], cfl_red<D, P>(smem, a.cells_per_block), cmax, vmax);
}

template <int D, int P>
size_t cfl_lds_bytes(int C, int nt)
{
    constexpr int NAP = Pad<P>::PP * ipow(P, D - 1);   // padded per-cell array
    return sizeof(double) * ((size_t)2 * C * (D + 2) * NAP + 2 * (size_t)nt);
}

// ---------------------------------------------------------------------------
// positivity limiter (Sec. 4.2), FP64 on the FP64 state
// ---------------------------------------------------------------------------
//
// One block = C consecutive cells.  The conserved fields are evaluated on the
// extended grid of E = p + 2 nodes per axis (-1, the p Gauss nodes, +1) by one
// E x p operator pass per axis; the limiter points are the grid points with at
// most one coordinate at -1 or +1 (the volume Gauss points and the Gauss
// points of the 2d faces).  Per cell: rho_min over the points; if below
// rho_bottom = 1e-6 rho_bar the weights of degree >= 1 of every field get the
// factor theta = (rho_bar - rho_bottom) / (rho_bar - rho_min); then theta is
// halved while the pressure of u_bar + theta (u - u_bar) at some point is
// below 1e-6 p_bar (at most kLimHalvings times, then the weights are zeroed).
// Cells whose mean density or pressure is not positive are left alone (the
// stage check flags them).  Only the cells that change are written.

constexpr int kLimHalvings = 60;

// 1D value of mode l at extended node j (0: -1, 1..P: Gauss, P+1: +1)
template <int P>
__device__ __forceinline__ double ext_val(const Tab<double> &t, int l, int j)
{
    return j == 0 ? t.em[l] : (j == P + 1 ? t.ep[l] : t.B[l][j - 1]);
}

template <int D, int P>
struct LimGeo {
    static constexpr int E = P + 2;
    static constexpr int NE = ipow(E, D);            // extended grid points per cell
    static constexpr int Fc = D + 2;
};

template <int D, int P>
__host__ __device__ constexpr size_t lim_lds_bytes(int C, int nt)
{
    // two ping-pong arrays [Fc][C][E^D], per-(cell, lane) partial minima,
    // per-cell theta / status
    return sizeof(double) * (2 * (size_t)(D + 2) * C * ipow(P + 2, D) + (size_t)nt + 2 * (size_t)C) + 16;
}

template <int D, int P, int PH>
__device__ __forceinline__ void limit_tile(const Phys &ph, const Geo &geo, double *__restrict__ w,
                                           unsigned char *smem, int C, long long tile)
{
    constexpr int E = LimGeo<D, P>::E, NE = LimGeo<D, P>::NE, Fc = D + 2;
    constexpr int NP = ipow(P, D);
    constexpr int F = Fld<D, PH>::F;
    constexpr bool PN = Fld<D, PH>::PN;
    using BS = Basis<D, P, PN>;
    constexpr int NM = BS::NM;
    constexpr int FNP = F * NM;
    const Tab<double> &tb = TabSel<double>::get(P);
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = tile * C;
    const int CN = C * NE;                           // one field of the tile
    double *X = (double *)smem;                      // [Fc][C][NE]
    double *Y = X + (size_t)Fc * CN;
    double *red = Y + (size_t)Fc * CN;               // [nt]
    double *theta = red + nt;                        // [C]
    double *stat = theta + C;                        // [C]: 1 = still halving
    int *more_flag = (int *)(stat + C);              // some cell still halving
    // pass along x: line (f, c, t), t = transverse mode (l_y[, l_z]); output
    // index ((f C + c) p^(d-1) + t) E + j_x
    constexpr int K = NP / P;
    for (int q = tid; q < Fc * C * K; q += nt) {
        const int arr = q / K, t = q - arr * K;
        const int f = arr / C, c = arr - f * C;
        long long cc = c0 + c;
        if (cc >= NC) cc = NC - 1;
        const int ly = t % P, lz = t / P;
        const double *src = w + cc * FNP + f * NM + BS::off(ly, lz);
        const int nl = BS::len(ly, lz);
        double x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = k < nl ? src[k] : 0.0;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) acc = fma(ext_val<P>(tb, k, j), x[k], acc);
            Y[q * E + j] = acc;
        }
    }
    __syncthreads();
    // pass along y: line (f, c, l_z, j_x): P values at stride E -> E values at
    // stride E; output ((f C + c) p^(d-2) + l_z) E^2 + j_y E + j_x
    constexpr int KZ = (D == 3) ? P : 1;
    for (int q = tid; q < Fc * C * KZ * E; q += nt) {
        const int jx = q % E, r = q / E;             // r = (f C + c) KZ + l_z
        const double *in = Y + (size_t)r * P * E + jx;
        double x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = in[k * E];
        double *out = X + (size_t)r * E * E + jx;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) acc = fma(ext_val<P>(tb, k, j), x[k], acc);
            out[j * E] = acc;
        }
    }
    __syncthreads();
    const double *V = X;
    if (D == 3) {
        // pass along z: line (f, c, j_y, j_x): P values at stride E^2
        for (int q = tid; q < Fc * C * E * E; q += nt) {
            const int jxy = q % (E * E), arr = q / (E * E);
            const double *in = X + (size_t)arr * P * E * E + jxy;
            double x[P];
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] = in[k * E * E];
            double *out = Y + (size_t)arr * NE + jxy;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) acc = fma(ext_val<P>(tb, k, j), x[k], acc);
                out[j * E * E] = acc;
            }
        }
        __syncthreads();
        V = Y;
    }
    // lanes per cell for the per-cell minima (block size is a multiple of 64)
    const int S = nt / C > 0 ? nt / C : 1;
    const int cl = tid / S, sl = tid - cl * S;
    auto is_point = [&](int j) {
        int ends = 0, r = j;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const int jb = r % E;
            r /= E;
            ends += (jb == 0 || jb == E - 1) ? 1 : 0;
        }
        return ends <= 1;
    };
    auto cell_means = [&](int c, double *um) {
        long long cc = c0 + c;
        if (cc >= NC) cc = NC - 1;
#pragma unroll
        for (int f = 0; f < Fc; ++f) um[f] = w[cc * FNP + f * NM];
    };
    // minimum in which NaN counts as lower than anything (a NaN pressure must
    // be limited)
    auto lowest = [](double a, double b) { return (b >= a || a != a) ? a : b; };
    auto pres = [&](const double *u) {
        const double rho = u[0];
        double v2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = u[1 + i] / rho;
            v2 += v * v;
        }
        return (ph.gamma - 1.0) * (u[D + 1] - 0.5 * rho * v2);
    };
    // density minima
    double rmin = 1.0 / 0.0;
    if (cl < C)
        for (int j = sl; j < NE; j += S)
            if (is_point(j)) rmin = fmin(rmin, V[cl * NE + j]);
    red[tid] = rmin;
    __syncthreads();
    for (int c = tid; c < C; c += nt) {
        double m = red[c * S];
        for (int k = 1; k < S; ++k) m = fmin(m, red[c * S + k]);
        double um[Fc];
        cell_means(c, um);
        const double rbar = um[0], pbar = pres(um);
        double th = 1.0, st = 0.0;
        if (rbar > 0.0 && pbar > 0.0 && c0 + c < NC) {
            const double rb = 1e-6 * rbar;
            if (m < rb) th = (rbar - rb) / (rbar - m);
            st = 1.0;                                // pressure stage to do
        }
        theta[c] = th;
        stat[c] = st;
    }
    __syncthreads();
    // pressure: halve theta while some point is below p_bottom (block-uniform
    // loop, at most kLimHalvings + 1 evaluations)
    for (int it = 0; it <= kLimHalvings; ++it) {
        double pmin = 1.0 / 0.0;
        if (cl < C && stat[cl] != 0.0) {
            double um[Fc];
            cell_means(cl, um);
            const double th = theta[cl];
            for (int j = sl; j < NE; j += S)
                if (is_point(j)) {
                    double u[Fc];
#pragma unroll
                    for (int f = 0; f < Fc; ++f) u[f] = um[f] + th * (V[(f * C + cl) * NE + j] - um[f]);
                    const double pk = pres(u);
                    pmin = lowest(pmin, pk);
                }
        }
        red[tid] = pmin;
        if (tid == 0) *more_flag = 0;
        __syncthreads();
        for (int c = tid; c < C; c += nt) {
            if (stat[c] == 0.0) continue;
            double m = red[c * S];
            for (int k = 1; k < S; ++k) m = lowest(m, red[c * S + k]);
            double um[Fc];
            cell_means(c, um);
            const double pb = 1e-6 * pres(um);
            if (m >= pb) {
                stat[c] = 0.0;
            } else if (it == kLimHalvings) {
                theta[c] = 0.0;
                stat[c] = 0.0;
            } else {
                theta[c] *= 0.5;
                *more_flag = 1;
            }
        }
        // block-uniform continuation: any cell still halving
        __syncthreads();
        const int more = *more_flag;
        __syncthreads();                             // read before the next reset
        if (!more) break;
    }
    // write the limited cells: weights of degree >= 1 of every field
    for (int q = tid; q < C * F * NM; q += nt) {
        const int c = q / (F * NM), r = q - c * (F * NM);
        if (r % NM == 0) continue;                   // the mean
        const double th = theta[c];
        const long long cc = c0 + c;
        if (th < 1.0 && cc < NC) w[cc * FNP + r] *= th;
    }
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(512) limit_kernel(Phys ph, Geo geo, double *w, int C)
{
    extern __shared__ __align__(16) unsigned char smem[];
    limit_tile<D, P, PH>(ph, geo, w, smem, C, blockIdx.x);
}

// ---------------------------------------------------------------------------
// fixed-tile volume kernels of the tuned table
// ---------------------------------------------------------------------------

// Entry I of the tuned table as a fixed-tile kernel of this (dim, precision)
// unit, or an empty record.  FO = 1 (forcing) variants exist for 3D entries.
template <int DIM, int PREC, typename T, size_t I, int FO>
FixedVol fixed_vol_entry()
{
    constexpr TileEntry e = kTiles[I];
    if constexpr (e.dim == DIM && e.prec == PREC && e.order >= 1 && e.order <= MAXP && e.phys >= 0 && e.phys <= 7 &&
                  e.vol_C > 0 && e.vol_T >= 64 && e.vol_T <= 512 && e.vol_T % 64 == 0 && (FO == 0 || DIM == 3))
        return FixedVol{e.order, e.phys, e.vol_C, e.vol_T, FO,
                        (const void *)&vol_kernel_fixed<DIM, e.order, T, e.phys, e.vol_C, e.vol_T, FO>,
                        FO == 0 ? (const void *)&vol_kernel_batched_fixed<DIM, e.order, T, e.phys, e.vol_C, e.vol_T>
                                : nullptr};
    else
        return FixedVol{0, 0, 0, 0, 0, nullptr, nullptr};
}

// Entry I of the tuned table as a fixed-tile face kernel, or an empty record.
template <int DIM, int PREC, typename T, size_t I>
FixedVol fixed_face_entry()
{
    constexpr TileEntry e = kTiles[I];
    if constexpr (e.dim == DIM && e.prec == PREC && e.order >= 1 && e.order <= MAXP && e.phys >= 0 && e.phys <= 7 &&
                  e.face_C > 0 && e.face_T >= 64 && e.face_T <= 512 && e.face_T % 64 == 0)
        return FixedVol{e.order, e.phys, e.face_C, e.face_T, 0,
                        (const void *)&face_kernel_fixed<DIM, e.order, T, e.phys, e.face_C, e.face_T>,
                        (const void *)&face_kernel_batched_fixed<DIM, e.order, T, e.phys, e.face_C, e.face_T>};
    else
        return FixedVol{0, 0, 0, 0, 0, nullptr, nullptr};
}

template <int DIM, int PREC, typename T, size_t... I>
const void *find_fixed_face(int order, int phys, int C, int NT, int batched, std::index_sequence<I...>)
{
    static const FixedVol tab[] = {fixed_face_entry<DIM, PREC, T, I>()..., FixedVol{0, 0, 0, 0, 0, nullptr, nullptr}};
    for (const FixedVol &f : tab)
        if (f.fn && f.order == order && f.phys == phys && f.C == C && f.NT == NT) return batched ? f.fnb : f.fn;
    return nullptr;
}

template <int DIM, int PREC, typename T, size_t... I>
const void *find_fixed_vol(int order, int phys, int C, int NT, int forced, int batched,
                           std::index_sequence<I...>)
{
    static const FixedVol tab[] = {fixed_vol_entry<DIM, PREC, T, I, 0>()...,
                                   fixed_vol_entry<DIM, PREC, T, I, 1>()..., FixedVol{0, 0, 0, 0, 0, nullptr, nullptr}};
    for (const FixedVol &f : tab)
        if (f.fn && f.order == order && f.phys == phys && f.C == C && f.NT == NT && f.forced == forced)
            return batched ? f.fnb : f.fn;
    return nullptr;
}

}  // namespace dgk
