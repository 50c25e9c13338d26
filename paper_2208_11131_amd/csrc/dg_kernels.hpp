// dg_kernels.hpp -- HIP kernels of the DG right-hand side for gfx950.
//
// Included once by each instantiation unit (dg_inst_*.hip).  Each unit gets
// its own copy of the per-order tables in __constant__ memory (uploaded by
// the host runtime through the unit's dgk_upload_* entry).
//
// Work decomposition (one HIP thread block = a tile of whole cells or faces,
// all intermediate data in LDS):
//   face kernel    per face of direction a = blockIdx.y: traces of both
//                  cells, HLLC, and (viscous/AV) the interface recovery of
//                  Sec. 3.2 with the Navier-Stokes/AV flux; writes one
//                  single-valued flux per face point to the face buffer.
//   volume kernel  per cell: modal -> Gauss-point values by sum factorisation
//                  (one p x p operator per axis), collocation gradients,
//                  point fluxes and sources, D^T and the face lift in point
//                  space, point -> modal projection, prefactor 2^(1-d)/h,
//                  and the SSP-RK stage combination in FP64.
//   cfl kernel     maxima of c_s and |v| over all volume Gauss points.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_common.hpp"

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

enum { M_B = 0, M_BT = 1, M_D = 2, M_DT = 3, M_BD = 4 };

// Entry (k, i) of the operator applied by axis_pass: out_i = sum_k M(k, i) in_k.
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

// Apply a p x p operator along axis AX of ncell*nper arrays of p^DA entries.
// Array (c, f) starts at in + c*in_cs + f*p^DA (likewise out).  Each work item
// is one line along AX: p loads, p*p FMAs with table operands, p stores.
template <int P, int DA, int AX, typename T, int MAT, bool ACC>
__device__ __forceinline__ void axis_pass(const T *__restrict__ in, int in_cs, T *__restrict__ out, int out_cs,
                                          int ncell, int nper)
{
    constexpr int NA = ipow(P, DA);
    constexpr int NL = NA / P;
    constexpr int S = ipow(P, AX);
    const int nitems = ncell * nper * NL;
    for (int q = threadIdx.x; q < nitems; q += blockDim.x) {
        const int cf = q / NL;
        const int t = q - cf * NL;
        const int c = cf / nper;
        const int f = cf - c * nper;
        const int lo = t % S, hi = t / S;
        const int off = f * NA + lo + hi * S * P;
        const T *pi = in + c * in_cs + off;
        T *po = out + c * out_cs + off;
        T x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = pi[k * S];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            T acc = ACC ? po[i * S] : T(0);
#pragma unroll
            for (int k = 0; k < P; ++k) acc = fma(mat<P, T, MAT>(k, i), x[k], acc);
            po[i * S] = acc;
        }
    }
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

// HLLC flux (Toro ch. 10) with Davis wave-speed bounds.
template <int D, typename T>
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
        return;
    }
    if (SR <= T(0)) {
        euler_flux<D, T>(uR, R, a, F);
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
    const T fac = K.rho * (S - un) / (S - Ss);
    T us[D + 2];
    us[0] = fac;
#pragma unroll
    for (int i = 0; i < D; ++i) us[1 + i] = (i == a) ? fac * Ss : fac * K.v[i];
    us[D + 1] = fac * (u[D + 1] * K.ir + (Ss - un) * (Ss + K.p / (K.rho * (S - un))));
#pragma unroll
    for (int k = 0; k < D + 2; ++k) F[k] += S * (us[k] - u[k]);
}

// Navier-Stokes flux along axis a (added with a minus sign to the Euler flux):
// (0, Pi_{.a}, v.Pi_{.a} + chi (gamma-1) rho d_a e_int),
// Pi = nu rho (grad v + grad v^T - 2/3 div v I).  g[b][f]: d u_f / d x_b.
template <int D, typename T>
__device__ __forceinline__ void ns_flux(const T *u, const Prim<D, T> &s, const T (*g)[MAXF], int a, T gamma, T nu,
                                        T chi, T *fv)
{
    T dv[D][D];
#pragma unroll
    for (int b = 0; b < D; ++b)
#pragma unroll
        for (int i = 0; i < D; ++i) dv[i][b] = (g[b][1 + i] - s.v[i] * g[b][0]) * s.ir;
    T div = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) div += dv[i][i];
    T de = (g[a][D + 1] - u[D + 1] * s.ir * g[a][0]) * s.ir;
#pragma unroll
    for (int i = 0; i < D; ++i) de -= s.v[i] * dv[i][a];
    const T nr = nu * s.rho;
    fv[0] = T(0);
    T vp = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const T pi = nr * (dv[i][a] + dv[a][i] - (i == a ? T(2.0 / 3.0) * div : T(0)));
        fv[1 + i] = pi;
        vp += s.v[i] * pi;
    }
    fv[D + 1] = vp + chi * (gamma - T(1)) * s.rho * de;
}

template <typename T>
__device__ __forceinline__ T clamp_alpha(T al, T amax)
{
    return al < T(0) ? T(0) : (al > amax ? amax : al);
}

// ---------------------------------------------------------------------------
// face kernel
// ---------------------------------------------------------------------------

// Cell index of the lower (side 0) or upper (side 1) cell of face fi of
// direction ax, and whether it is a mirrored ghost.
__device__ __forceinline__ long long face_cell(const Geo &g, int ax, long long fi, int side, bool &mirror)
{
    int co[3] = {0, 0, 0};
    long long r = fi;
    for (int b = 0; b < 3; ++b) {
        const int nb = (b == ax) ? g.nf[b] : g.n[b];
        co[b] = (int)(r % nb);
        r /= nb;
    }
    mirror = false;
    int ia = co[ax] - (side == 0 ? 1 : 0);
    if (g.bc[ax] == 0) {
        if (ia < 0) ia += g.n[ax];
    } else {
        if (ia < 0) {
            ia = 0;
            mirror = true;
        } else if (ia >= g.n[ax]) {
            ia = g.n[ax] - 1;
            mirror = true;
        }
    }
    co[ax] = ia;
    return co[0] + (long long)g.n[0] * (co[1] + (long long)g.n[1] * co[2]);
}

template <int D, int P, int AX, typename T, bool GRAD>
__device__ __forceinline__ void face_body(const Phys &ph, const Geo &geo, const FaceArgs &a, unsigned char *smem)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;          // face points (and transverse modes)
    const int Fc = D + 2;
    const int F = Fc + ph.av_on;
    const int C = a.faces_per_block;
    const long long nfc = geo.nfaces[AX];
    const long long f0 = (long long)blockIdx.x * C;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Q = C * F * K;
    const int NA = GRAD ? 4 : 2;

    long long *cellidx = (long long *)smem;               // [2][C]
    int *mir = (int *)(cellidx + 2 * C);                  // [2][C]
    T *base = (T *)(smem + ((2 * C * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16);
    T *WL = base;                                         // [C][F][NP]
    T *WR = WL + C * F * NP;
    T *A = WR + C * F * NP;                               // [NA][C][F][K]
    T *Sx = (P >= 3) ? WL : (A + NA * Q);                 // scratch [6][C][F][K]

    for (int e = tid; e < 2 * C; e += nt) {
        const int side = e / C, c = e - side * C;
        long long fi = f0 + c;
        if (fi >= nfc) fi = nfc - 1;
        bool m;
        cellidx[e] = face_cell(geo, AX, fi, side, m);
        mir[e] = m ? 1 : 0;
    }
    __syncthreads();
    for (int i = tid; i < 2 * C * F * NP; i += nt) {
        const int side = i / (C * F * NP);
        const int r = i - side * C * F * NP;
        const int c = r / (F * NP);
        const int e = r - c * F * NP;
        double v = a.w[cellidx[side * C + c] * (long long)(F * NP) + e];
        if (mir[side * C + c]) {
            const int m = e % NP;
            const int la = (m / ipow(P, AX)) % P;
            if (la & 1) v = -v;
        }
        (side ? WR : WL)[r] = (T)v;
    }
    __syncthreads();

    // normal contraction: traces (and recovery partial sums) per transverse mode
    {
        constexpr int S = ipow(P, AX);
        const Tab<T> &tb = TabSel<T>::get(P);
        for (int q = tid; q < C * F * K; q += nt) {
            const int cf = q / K;
            const int t = q - cf * K;
            const int lo = t % S, hi = t / S;
            const int off = cf * NP + lo + hi * S * P;
            T xl[P], xr[P];
#pragma unroll
            for (int m = 0; m < P; ++m) {
                xl[m] = WL[off + m * S];
                xr[m] = WR[off + m * S];
            }
            T tl = T(0), tr = T(0);
#pragma unroll
            for (int m = 0; m < P; ++m) {
                tl = fma(tb.ep[m], xl[m], tl);
                tr = fma(tb.em[m], xr[m], tr);
            }
            A[0 * Q + q] = tl;
            A[1 * Q + q] = tr;
            if (GRAD) {
                T rv = T(0), rn = T(0);
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    rv = fma(tb.rvL[m], xl[m], rv);
                    rv = fma(tb.rvR[m], xr[m], rv);
                    rn = fma(tb.rdL[m], xl[m], rn);
                    rn = fma(tb.rdR[m], xr[m], rn);
                }
                A[2 * Q + q] = rv;
                A[3 * Q + q] = rn;
            }
        }
    }
    __syncthreads();

    // transverse transforms to the face Gauss points
    const T *tLp, *tRp, *utp = nullptr, *rnp = nullptr, *d1p = nullptr, *d2p = nullptr;
    if (D == 2) {
        axis_pass<P, 1, 0, T, M_B, false>(A, K, Sx, K, NA * C * F, 1);
        if (GRAD) axis_pass<P, 1, 0, T, M_BD, false>(A + 2 * Q, K, Sx + 4 * Q, K, C * F, 1);
        __syncthreads();
        tLp = Sx;
        tRp = Sx + Q;
        utp = Sx + 2 * Q;
        rnp = Sx + 3 * Q;
        d1p = Sx + 4 * Q;
    } else {
        axis_pass<P, 2, 0, T, M_B, false>(A, K, Sx, K, NA * C * F, 1);
        if (GRAD) axis_pass<P, 2, 0, T, M_BD, false>(A + 2 * Q, K, Sx + 4 * Q, K, C * F, 1);
        __syncthreads();
        axis_pass<P, 2, 1, T, M_B, false>(Sx, K, A, K, NA * C * F, 1);
        if (GRAD) axis_pass<P, 2, 1, T, M_BD, false>(Sx + 2 * Q, K, Sx + 5 * Q, K, C * F, 1);
        __syncthreads();
        if (GRAD) {
            axis_pass<P, 2, 1, T, M_B, false>(Sx + 4 * Q, K, Sx, K, C * F, 1);
            __syncthreads();
        }
        tLp = A;
        tRp = A + Q;
        utp = A + 2 * Q;
        rnp = A + 3 * Q;
        d1p = Sx;
        d2p = Sx + 5 * Q;
    }

    // point fluxes
    const T gamma = (T)ph.gamma;
    const Tab<T> &tb = TabSel<T>::get(P);
    T *fb = (T *)a.fb + geo.fb_off[AX];
    for (int q = tid; q < C * K; q += nt) {
        const int c = q / K, k = q - c * K;
        const long long fi = f0 + c;
        if (fi >= nfc) continue;
        T uL[D + 2], uR[D + 2], Fh[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) {
            uL[f] = tLp[(c * F + f) * K + k];
            uR[f] = tRp[(c * F + f) * K + k];
        }
        hllc<D, T>(uL, uR, AX, gamma, Fh);
        if (GRAD) {
            T ut[MAXF];
            T g[D][MAXF];
            constexpr int T1 = (AX == 0) ? 1 : 0;             // transverse axes, ascending
            constexpr int T2 = (D == 3) ? ((AX == 2) ? 1 : 2) : 0;
#pragma unroll
            for (int f = 0; f < D + 3; ++f) {
                if (f < F) {
                    const int idx = (c * F + f) * K + k;
                    ut[f] = utp[idx];
                    g[AX][f] = rnp[idx] * (T)ph.inv_fh;
                    g[T1][f] = d1p[idx] * (T)ph.two_over_h;
                    if (D == 3) g[T2][f] = d2p[idx] * (T)ph.two_over_h;
                }
            }
            const Prim<D, T> s = primitives<D, T>(ut, gamma);
            if (ph.ns_on) {
                T fv[D + 2];
                ns_flux<D, T>(ut, s, g, AX, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
                for (int f = 0; f < D + 2; ++f) Fh[f] -= fv[f];
            }
            if (ph.av_on) {
                const T cs = sqrt(gamma * s.p * s.ir);
                const T eps = (T)ph.av_scale * clamp_alpha(ut[D + 2], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
#pragma unroll
                for (int f = 0; f < D + 2; ++f) Fh[f] -= eps * g[AX][f];
            }
        }
        T gk = tb.g[k % P];
        if (D == 3) gk *= tb.g[k / P];
        T *dst = fb + fi * (long long)(Fc * K) + k;
#pragma unroll
        for (int f = 0; f < D + 2; ++f) dst[f * K] = gk * Fh[f];
    }
}

template <int D, int P, typename T, bool GRAD>
__global__ void __launch_bounds__(512) face_kernel(Phys ph, Geo geo, FaceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int ax = blockIdx.y;
    if ((long long)blockIdx.x * a.faces_per_block >= geo.nfaces[ax]) return;
    if (ax == 0)
        face_body<D, P, 0, T, GRAD>(ph, geo, a, smem);
    else if (ax == 1)
        face_body<D, P, 1, T, GRAD>(ph, geo, a, smem);
    else if (D == 3)
        face_body<D, P, (D == 3 ? 2 : 0), T, GRAD>(ph, geo, a, smem);
}

// LDS bytes of the face kernel for C faces per block: header, the two cells'
// coefficients W (2 C F p^d), the contraction results A (NA C F p^(d-1)) and
// a scratch of 6 C F p^(d-1) that overlays W when p >= 3 (W is dead after
// the normal contraction).
template <int D, int P, typename T, bool GRAD>
size_t face_lds_bytes(int C, int F)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    const size_t hdr = ((2 * C * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16;
    const size_t Q = (size_t)C * F * K;
    const size_t W = 2 * (size_t)C * F * NP;
    const size_t NA = GRAD ? 4 : 2;
    const size_t tot = W + NA * Q + (P >= 3 ? 0 : 6 * Q);
    return hdr + sizeof(T) * tot;
}

// ---------------------------------------------------------------------------
// volume kernel
// ---------------------------------------------------------------------------

template <int D, int P, typename T, bool GRAD>
__global__ void __launch_bounds__(512) vol_kernel(Phys ph, Geo geo, VolArgs a)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Fc = D + 2;
    const int F = Fc + ph.av_on;
    const int Fx = F + (a.forcing ? D : 0);
    const int C = a.cells_per_block;
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = (long long)blockIdx.x * C;
    const int cs_x = Fx * NP;                 // per-cell stride of X0/X1
    const int cs_g = D * F * NP;              // per-cell stride of G

    double *cellv = (double *)smem;           // [C][2]: wiggle source, new mean checks
    int *blkflag = (int *)(cellv + 2 * C);
    T *X0 = (T *)(smem + ((2 * C * sizeof(double) + sizeof(int) + 15) / 16) * 16);
    T *X1 = X0 + C * cs_x;
    T *G = X1 + C * cs_x;
    const Tab<T> &tb = TabSel<T>::get(P);

    // 1. load the tile's weights (and forcing coefficients)
    const long long gbase = c0 * F * NP, gend = NC * F * NP;
    for (int i = tid; i < C * F * NP; i += nt) {
        const int c = i / (F * NP), r = i - c * (F * NP);
        long long gi = gbase + i;
        if (gi >= gend) gi = (NC - 1) * F * NP + r;
        X0[c * cs_x + r] = (T)a.cur[gi];
    }
    if (a.forcing) {
        for (int i = tid; i < C * D * NP; i += nt) {
            const int c = i / (D * NP), r = i - c * (D * NP);
            long long cc = c0 + c;
            if (cc >= NC) cc = NC - 1;
            X0[c * cs_x + F * NP + r] = (T)a.forcing[cc * D * NP + r];
        }
    }
    if (tid == 0) *blkflag = 0;
    for (int cl = tid; ph.av_on && cl < C; cl += nt) {
        // sensor S of the current state and the wiggle source (Sec. 4.1)
        long long cc = c0 + cl;
        if (cc >= NC) cc = NC - 1;
        const double *wr = a.cur + cc * F * NP;
        double all = 0.0, top = 0.0;
        for (int m = 0; m < NP; ++m) {
            const double x = wr[m];
            all += x * x;
            bool t = false;
            int r = m;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                t = t || (r % P == P - 1);
                r /= P;
            }
            if (t) top += x * x;
        }
        const double S = all > 0.0 ? top / all : 0.0;
        const double Rp = a.R_prev ? a.R_prev[cc] : 0.0;
        cellv[2 * cl] = (S > ph.s_thr) ? ph.f_w * fmax(0.0, Rp) : 0.0;
    }
    __syncthreads();

    // 2. point values of all fields: one operator pass per axis
    axis_pass<P, D, 0, T, M_B, false>(X0, cs_x, X1, cs_x, C, Fx);
    __syncthreads();
    axis_pass<P, D, 1, T, M_B, false>(X1, cs_x, X0, cs_x, C, Fx);
    __syncthreads();
    if (D == 3) {
        axis_pass<P, D, (D == 3 ? 2 : 0), T, M_B, false>(X0, cs_x, X1, cs_x, C, Fx);
        __syncthreads();
    }
    T *U = (D == 3) ? X1 : X0;
    T *Wk = (D == 3) ? X0 : X1;

    // 3. collocation gradients d/dxi of the stored fields
    if (GRAD) {
        axis_pass<P, D, 0, T, M_D, false>(U, cs_x, G, cs_g, C, F);
        axis_pass<P, D, 1, T, M_D, false>(U, cs_x, G + F * NP, cs_g, C, F);
        if (D == 3) axis_pass<P, D, (D == 3 ? 2 : 0), T, M_D, false>(U, cs_x, G + 2 * F * NP, cs_g, C, F);
        __syncthreads();
    }

    // 4. point fluxes (weighted by the volume Gauss weights) and sources
    const T gamma = (T)ph.gamma;
    for (int q = tid; q < C * NP; q += nt) {
        const int c = q / NP, j = q - c * NP;
        T u[MAXF];
#pragma unroll
        for (int f = 0; f < 2 * D + 3; ++f)
            if (f < Fx) u[f] = U[c * cs_x + f * NP + j];
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
                for (int f = 0; f < D + 3; ++f)
                    if (f < F) g[b][f] = G[c * cs_g + (b * F + f) * NP + j] * (T)ph.two_over_h;
        }
        T eps = T(0), cs = T(0);
        if (ph.av_on) {
            cs = sqrt(gamma * s.p * s.ir);
            eps = (T)ph.av_scale * clamp_alpha(u[Fc], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
        }
#pragma unroll
        for (int b = 0; b < D; ++b) {
            T fl[D + 2];
            euler_flux<D, T>(u, s, b, fl);
            if (GRAD && ph.ns_on) {
                T fv[D + 2];
                ns_flux<D, T>(u, s, g, b, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
                for (int f = 0; f < D + 2; ++f) fl[f] -= fv[f];
            }
            if (GRAD && ph.av_on) {
#pragma unroll
                for (int f = 0; f < D + 2; ++f) fl[f] -= eps * g[b][f];
            }
#pragma unroll
            for (int f = 0; f < D + 2; ++f) G[c * cs_g + (b * F + f) * NP + j] = wq * fl[f];
        }
        // sources, scaled to the common prefactor: Q = (h/2) w_j src
        const T hw = (T)ph.half_h * wq;
        T src[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) src[f] = T(0);
        if (a.forcing) {
            // the forcing fields follow the stored ones: index F = Fc + av_on
            T sf[D];
#pragma unroll
            for (int i = 0; i < D; ++i) sf[i] = ph.av_on ? u[D + 3 + i] : u[D + 2 + i];
            T sv = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                src[1 + i] = s.rho * sf[i];
                sv += sf[i] * u[1 + i];
            }
            src[D + 1] = sv;
        }
#pragma unroll
        for (int f = 0; f < D + 2; ++f) U[c * cs_x + f * NP + j] = hw * src[f];
        if (ph.av_on) {
            T div = T(0);
            if (GRAD) {
#pragma unroll
                for (int i = 0; i < D; ++i) div += (g[i][1 + i] - s.v[i] * g[i][0]) * s.ir;
            }
            const T asrc = (T)ph.f_v * fmax(T(0), -div) + (T)cellv[2 * c] - u[Fc] * cs * (T)ph.sink;
            U[c * cs_x + Fc * NP + j] = hw * asrc;
        }
    }
    __syncthreads();

    // 5. Q += sum_a D_a^T (w f_a)
    axis_pass<P, D, 0, T, M_DT, true>(G, cs_g, U, cs_x, C, Fc);
    __syncthreads();
    axis_pass<P, D, 1, T, M_DT, true>(G + F * NP, cs_g, U, cs_x, C, Fc);
    __syncthreads();
    if (D == 3) {
        axis_pass<P, D, (D == 3 ? 2 : 0), T, M_DT, true>(G + 2 * F * NP, cs_g, U, cs_x, C, Fc);
        __syncthreads();
    }

    // 6. surface lift in point space: Q(i, k) += L_i(-1) F_lower(k) - L_i(+1) F_upper(k)
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const int S = (ax == 0) ? 1 : (ax == 1 ? P : P * P);
        const T *fb = (const T *)a.fb + geo.fb_off[ax];
        for (int q = tid; q < C * Fc * K; q += nt) {
            const int c = q / (Fc * K);
            const int r = q - c * (Fc * K);
            const int f = r / K, k = r - f * K;
            long long cc = c0 + c;
            if (cc >= NC) cc = NC - 1;
            // face indices of the lower and upper face of cell cc along ax
            int co[3] = {0, 0, 0};
            long long t = cc;
            for (int b = 0; b < 3; ++b) {
                co[b] = (int)(t % geo.n[b]);
                t /= geo.n[b];
            }
            const int nfa = geo.nf[ax];
            long long flo = 0, fhi = 0, mul = 1;
            for (int b = 0; b < 3; ++b) {
                const int nb = (b == ax) ? nfa : geo.n[b];
                int ilo = co[b], ihi = co[b];
                if (b == ax) {
                    ihi = co[b] + 1;
                    if (ihi >= nfa) ihi -= nfa;    // periodic wrap (outflow has nf = n + 1)
                }
                flo += ilo * mul;
                fhi += ihi * mul;
                mul *= nb;
            }
            const T Fl = fb[flo * (Fc * K) + f * K + k];
            const T Fu = fb[fhi * (Fc * K) + f * K + k];
            const int lo = k % S, hi = k / S;
            T *po = U + c * cs_x + f * NP + lo + hi * S * P;
#pragma unroll
            for (int i = 0; i < P; ++i) po[i * S] += tb.Lm[i] * Fl - tb.Lp[i] * Fu;
        }
        __syncthreads();
    }

    // 7. point -> modal projection of every stored field
    axis_pass<P, D, 0, T, M_BT, false>(U, cs_x, Wk, cs_x, C, F);
    __syncthreads();
    axis_pass<P, D, 1, T, M_BT, false>(Wk, cs_x, U, cs_x, C, F);
    __syncthreads();
    if (D == 3) {
        axis_pass<P, D, (D == 3 ? 2 : 0), T, M_BT, false>(U, cs_x, Wk, cs_x, C, F);
        __syncthreads();
    }
    const T *V = (D == 3) ? Wk : U;

    // 8. RK combination in FP64 and write-back
    const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
    const double pref = ph.pref;
    int bad = 0;
    for (int i = tid; i < C * F * NP; i += nt) {
        const int c = i / (F * NP), r = i - c * (F * NP);
        const long long gi = gbase + i;
        if (gi >= gend) continue;
        const double L = pref * (double)V[c * cs_x + r];
        const double cur = a.cur[gi];
        double o = a.c_cur * cur + a.c_L * dt * L;
        if (a.base) o += a.c_base * a.base[gi];
        double o2 = 0.0;
        if (a.out2) {
            o2 = a.d_cur * cur + a.d_L * dt * L;
            if (a.x2) o2 += a.d_x2 * a.x2[gi];
        }
        a.out[gi] = o;
        if (a.out2) a.out2[gi] = o2;
        if (!isfinite(o)) bad |= 2;
    }
    if (bad) atomicOr(blkflag, bad);
    __syncthreads();

    // 9. per-cell checks (mean pressure) and, at stage 1, d ln S / dt
    for (int cl = tid; cl < C; cl += nt) {
        const long long cc = c0 + cl;
        if (cc < NC) {
            const double *o = a.out + cc * F * NP;
            const double rho = o[0];
            double m2 = 0.0;
            for (int i = 0; i < D; ++i) m2 += o[(1 + i) * NP] * o[(1 + i) * NP];
            const double pm = (ph.gamma - 1.0) * (o[(D + 1) * NP] - 0.5 * m2 / rho);
            if (a.check && !(rho > 0.0 && pm > 0.0)) atomicOr(blkflag, 1);
            if (a.R_out && ph.av_on) {
                const double *wr = a.cur + cc * F * NP;
                double A = 0.0, Tt = 0.0, ad = 0.0, td = 0.0;
                for (int m = 0; m < NP; ++m) {
                    const double x = wr[m];
                    const double xd = pref * (double)V[cl * cs_x + m];
                    A += x * x;
                    ad += x * xd;
                    bool t = false;
                    int r = m;
                    for (int b = 0; b < D; ++b) {
                        t = t || (r % P == P - 1);
                        r /= P;
                    }
                    if (t) {
                        Tt += x * x;
                        td += x * xd;
                    }
                }
                double R = 0.0;
                // rate kept only above the onset threshold (below it S is noise)
                if (A > 0.0 && Tt > 0.0 && Tt / A > ph.s_thr) {
                    const double S = Tt / A;
                    const double Sdot = 2.0 * (td * A - Tt * ad) / (A * A);
                    R = Sdot / S;
                }
                a.R_out[cc] = R;
            }
        }
    }
    __syncthreads();
    if (tid == 0 && *blkflag && a.flag) atomicOr(a.flag, *blkflag);
}

template <int D, int P, typename T>
size_t vol_lds_bytes(int C, int F, int Fx)
{
    constexpr int NP = ipow(P, D);
    const size_t hdr = ((2 * C * sizeof(double) + sizeof(int) + 15) / 16) * 16;
    return hdr + sizeof(T) * ((size_t)2 * C * Fx * NP + (size_t)C * D * F * NP);
}

// ---------------------------------------------------------------------------
// CFL kernel: maxima of c_s and |v| over the volume Gauss points (eq. timestep)
// ---------------------------------------------------------------------------

template <int D, int P>
__global__ void __launch_bounds__(512) cfl_kernel(Phys ph, Geo geo, CflArgs a)
{
    constexpr int NP = ipow(P, D);
    extern __shared__ __align__(16) unsigned char smem[];
    const int Fc = D + 2;
    const int F = Fc + ph.av_on;
    const int C = a.cells_per_block;
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = (long long)blockIdx.x * C;
    double *X0 = (double *)smem;
    double *X1 = X0 + C * Fc * NP;
    double *red = X1 + C * Fc * NP;      // [2][nt]
    for (int i = tid; i < C * Fc * NP; i += nt) {
        const int c = i / (Fc * NP), r = i - c * (Fc * NP);
        long long cc = c0 + c;
        if (cc >= NC) cc = NC - 1;
        X0[i] = a.w[cc * F * NP + r];
    }
    __syncthreads();
    axis_pass<P, D, 0, double, M_B, false>(X0, Fc * NP, X1, Fc * NP, C, Fc);
    __syncthreads();
    axis_pass<P, D, 1, double, M_B, false>(X1, Fc * NP, X0, Fc * NP, C, Fc);
    __syncthreads();
    if (D == 3) {
        axis_pass<P, D, (D == 3 ? 2 : 0), double, M_B, false>(X0, Fc * NP, X1, Fc * NP, C, Fc);
        __syncthreads();
    }
    const double *U = (D == 3) ? X1 : X0;
    double cmax = 0.0, vmax = 0.0;
    for (int q = tid; q < C * NP; q += nt) {
        const int c = q / NP, j = q - c * NP;
        if (c0 + c >= NC) continue;
        double u[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) u[f] = U[c * Fc * NP + f * NP + j];
        const Prim<D, double> s = primitives<D, double>(u, ph.gamma);
        double v2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) v2 += s.v[i] * s.v[i];
        const double cs = sqrt(ph.gamma * s.p * s.ir);
        const double vm = sqrt(v2);
        // NaN-propagating maxima (a NaN makes the step size NaN)
        cmax = (cs > cmax || cs != cs) ? cs : cmax;
        vmax = (vm > vmax || vm != vm) ? vm : vmax;
    }
    red[tid] = cmax;
    red[nt + tid] = vmax;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double c2 = red[tid + s], v2 = red[nt + tid + s];
            if (c2 > red[tid] || c2 != c2) red[tid] = c2;
            if (v2 > red[nt + tid] || v2 != v2) red[nt + tid] = v2;
        }
        __syncthreads();
    }
    if (tid == 0) {
        // non-negative doubles order like their bit patterns
        atomicMax(&a.maxbits[0], (unsigned long long)__double_as_longlong(red[0]));
        atomicMax(&a.maxbits[1], (unsigned long long)__double_as_longlong(red[nt]));
    }
}

template <int D, int P>
size_t cfl_lds_bytes(int C, int nt)
{
    constexpr int NP = ipow(P, D);
    return sizeof(double) * ((size_t)2 * C * (D + 2) * NP + 2 * (size_t)nt);
}

}  // namespace dgk
