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

// Apply a p x p operator along axis AX of ncell*NPER arrays of p^DA entries.
// Array (c, f) starts at in + c*in_cs + f*p^DA (likewise out).  Each work item
// is one line along AX: p loads, p*p FMAs with table operands, p stores.
template <int P, int DA, int AX, typename T, int MAT, bool ACC, int NPER>
__device__ __forceinline__ void axis_pass(const T *__restrict__ in, int in_cs, T *__restrict__ out, int out_cs,
                                          int ncell)
{
    constexpr int NA = ipow(P, DA);
    constexpr int NL = NA / P;
    constexpr int S = ipow(P, AX);
    const int nitems = ncell * NPER * NL;
    for (int q = threadIdx.x; q < nitems; q += blockDim.x) {
        const int cf = q / NL;
        const int t = q - cf * NL;
        const int c = cf / NPER;
        const int f = cf - c * NPER;
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

// Apply a p x p operator along axis AX of narr contiguous arrays of p^DA
// entries.  Line q starts at (q / S) * S * p + q % S (S = p^AX): a couple of
// integer operations per line; p loads, p*p FMAs with table operands, p stores.
template <int P, int DA, int AX, typename T, int MAT, bool ACC>
__device__ __forceinline__ void line_pass(const T *__restrict__ in, T *__restrict__ out, int narr)
{
    constexpr int NA = ipow(P, DA);
    constexpr int S = ipow(P, AX);
    const int nitems = narr * (NA / P);
    for (int q = threadIdx.x; q < nitems; q += blockDim.x) {
        const int off = (q / S) * (S * P) + (q % S);
        const T *pi = in + off;
        T *po = out + off;
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

// Fields per physics variant: PH = 0 Euler, 1 Navier-Stokes, 2 artificial
// viscosity (alpha field; Navier-Stokes terms switched at run time).
template <int D, int PH>
struct Fld {
    static constexpr int Fc = D + 2;
    static constexpr int F = D + 2 + (PH == 2 ? 1 : 0);
    static constexpr bool GRAD = PH > 0;
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
//
// One block computes a pencil of C consecutive faces of direction AX (fixed
// transverse coordinates).  It loads the C + 1 cells that these faces
// separate once, so every cell is read about once per direction.

template <int D, int P, int AX, typename T, int PH>
__device__ __forceinline__ void face_body(const Phys &ph, const Geo &geo, const FaceArgs &a, unsigned char *smem,
                                          long long pen_id)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;          // face points (and transverse modes)
    constexpr int Fc = Fld<D, PH>::Fc;
    constexpr int F = Fld<D, PH>::F;
    constexpr bool GRAD = Fld<D, PH>::GRAD;
    constexpr int FNP = F * NP;
    constexpr int NA = GRAD ? 4 : 2;
    constexpr int S = ipow(P, AX);
    const int C = a.faces_per_block;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Q = C * F * K;
    const int na = geo.n[AX], nfa = geo.nf[AX];
    const int npl = (nfa + C - 1) / C;
    const long long line = pen_id / npl;
    const int a0 = (int)(pen_id - line * npl) * C;
    const int nface = min(C, nfa - a0);
    int co[3] = {0, 0, 0};
    {
        long long r = line;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (b != AX) {
                co[b] = (int)(r % geo.n[b]);
                r /= geo.n[b];
            }
    }

    long long *cellidx = (long long *)smem;               // [C+1]
    int *mir = (int *)(cellidx + (C + 1));                // [C+1]
    T *W = (T *)(smem + (((C + 1) * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16);   // [C+1][F][NP]
    T *A = W + (C + 1) * FNP;                             // [NA][C][F][K]
    T *Sx = ((C + 1) * FNP >= 5 * Q) ? W : (A + NA * Q);  // scratch [5][C][F][K]

    for (int s = tid; s <= C; s += nt) {
        int ca = a0 + s - 1;
        int m = 0;
        if (geo.bc[AX] == 0) {
            ca = ((ca % na) + na) % na;   // pencils may be longer than the axis
        } else {
            if (ca < 0) {
                ca = 0;
                m = 1;
            } else if (ca >= na) {
                ca = na - 1;
                m = 1;
            }
        }
        int cc[3] = {co[0], co[1], co[2]};
        cc[AX] = ca;
        cellidx[s] = cc[0] + (long long)geo.n[0] * (cc[1] + (long long)geo.n[1] * cc[2]);
        mir[s] = m;
    }
    __syncthreads();
    for (int i = tid; i < (C + 1) * FNP; i += nt) {
        const int s = i / FNP, e = i - s * FNP;
        double v = a.w[cellidx[s] * FNP + e];
        if (mir[s] && (((e % NP) / S) % P) & 1) v = -v;
        W[i] = (T)v;
    }
    __syncthreads();

    // normal contraction: traces (and recovery partial sums) per transverse mode
    {
        const Tab<T> &tb = TabSel<T>::get(P);
        for (int q = tid; q < C * F * K; q += nt) {
            const int cf = q / K;
            const int t = q - cf * K;
            const int c = cf / F, f = cf - c * F;
            const int lo = t % S, hi = t / S;
            const int offL = c * FNP + f * NP + lo + hi * S * P;
            const int offR = offL + FNP;
            T xl[P], xr[P];
#pragma unroll
            for (int m = 0; m < P; ++m) {
                xl[m] = W[offL + m * S];
                xr[m] = W[offR + m * S];
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
        axis_pass<P, 1, 0, T, M_B, false, 1>(A, K, Sx, K, NA * C * F);
        if (GRAD) axis_pass<P, 1, 0, T, M_BD, false, 1>(A + 2 * Q, K, Sx + 4 * Q, K, C * F);
        __syncthreads();
        tLp = Sx;
        tRp = Sx + Q;
        utp = Sx + 2 * Q;
        rnp = Sx + 3 * Q;
        d1p = Sx + 4 * Q;
    } else {
        // (t1, t2) = transverse axes of the face in ascending order
        axis_pass<P, 2, 0, T, M_B, false, 1>(A, K, Sx, K, NA * C * F);
        if (GRAD) axis_pass<P, 2, 0, T, M_BD, false, 1>(A + 2 * Q, K, Sx + 4 * Q, K, C * F);
        __syncthreads();
        axis_pass<P, 2, 1, T, M_B, false, 1>(Sx, K, A, K, NA * C * F);
        __syncthreads();
        if (GRAD) {
            axis_pass<P, 2, 1, T, M_BD, false, 1>(Sx + 2 * Q, K, Sx, K, C * F);
            axis_pass<P, 2, 1, T, M_B, false, 1>(Sx + 4 * Q, K, Sx + Q, K, C * F);
            __syncthreads();
        }
        tLp = A;
        tRp = A + Q;
        utp = A + 2 * Q;
        rnp = A + 3 * Q;
        d2p = Sx;
        d1p = Sx + Q;
    }

    // point fluxes
    const T gamma = (T)ph.gamma;
    const Tab<T> &tb = TabSel<T>::get(P);
    T *fb = (T *)a.fb + geo.fb_off[AX];
    for (int q = tid; q < C * K; q += nt) {
        const int c = q / K, k = q - c * K;
        if (c >= nface) continue;
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
            for (int f = 0; f < F; ++f) {
                const int idx = (c * F + f) * K + k;
                ut[f] = utp[idx];
                g[AX][f] = rnp[idx] * (T)ph.inv_fh;
                g[T1][f] = d1p[idx] * (T)ph.two_over_h;
                if (D == 3) g[T2][f] = d2p[idx] * (T)ph.two_over_h;
            }
            const Prim<D, T> s = primitives<D, T>(ut, gamma);
            if (PH == 1 || ph.ns_on) {
                T fv[D + 2];
                ns_flux<D, T>(ut, s, g, AX, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
                for (int f = 0; f < D + 2; ++f) Fh[f] -= fv[f];
            }
            if (PH == 2) {
                const T cs = sqrt(gamma * s.p * s.ir);
                const T eps = (T)ph.av_scale * clamp_alpha(ut[D + 2], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
#pragma unroll
                for (int f = 0; f < D + 2; ++f) Fh[f] -= eps * g[AX][f];
            }
        }
        T gk = tb.g[k % P];
        if (D == 3) gk *= tb.g[k / P];
        int cf[3] = {co[0], co[1], co[2]};
        cf[AX] = a0 + c;
        const long long nd0 = (AX == 0) ? nfa : geo.n[0];
        const long long nd1 = (AX == 1) ? nfa : geo.n[1];
        const long long fi = cf[0] + nd0 * (cf[1] + nd1 * cf[2]);
        T *dst = fb + fi * (long long)(Fc * K) + k;
#pragma unroll
        for (int f = 0; f < D + 2; ++f) dst[f * K] = gk * Fh[f];
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

template <int D, int P, typename T, int PH>
__device__ __forceinline__ void face_dispatch(const Phys &ph, const Geo &geo, const FaceArgs &a, unsigned char *smem,
                                              int ax, long long pen)
{
    if (ax == 0)
        face_body<D, P, 0, T, PH>(ph, geo, a, smem, pen);
    else if (ax == 1)
        face_body<D, P, 1, T, PH>(ph, geo, a, smem, pen);
    else if (D == 3)
        face_body<D, P, (D == 3 ? 2 : 0), T, PH>(ph, geo, a, smem, pen);
}

template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) face_kernel(Phys ph, Geo geo, FaceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int ax = blockIdx.y;
    const unsigned bid = xcd_block(blockIdx.x, gridDim.x);
    if ((long long)bid >= pencils(geo, ax, a.faces_per_block)) return;
    face_dispatch<D, P, T, PH>(ph, geo, a, smem, ax, bid);
}

// Index of the box owning flat block b of a grouped launch (uniform scan).
__device__ __forceinline__ int owner_box(const BoxDesc *boxes, int nbox, long long b, int which)
{
    int i = 0;
    while (i + 1 < nbox && boxes[i + 1].start[which] <= b) ++i;
    return i;
}

// Grouped face kernel: every box of one (dim, order) group; flat block index
// -> (box, direction, pencil).
template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) face_kernel_batched(const BoxDesc *boxes, int nbox, int stage_cur)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = xcd_block(blockIdx.x, gridDim.x);
    const int i = owner_box(boxes, nbox, b, 1);
    const Phys ph = boxes[i].ph;
    const Geo geo = boxes[i].geo;
    FaceArgs a;
    a.w = boxes[i].reg[stage_cur];
    a.fb = boxes[i].fb;
    a.faces_per_block = boxes[i].faces_per_block;
    long long loc = b - boxes[i].start[1];
    for (int ax = 0; ax < D; ++ax) {
        const long long n = pencils(geo, ax, a.faces_per_block);
        if (loc < n) {
            face_dispatch<D, P, T, PH>(ph, geo, a, smem, ax, loc);
            return;
        }
        loc -= n;
    }
}

// LDS bytes of the face kernel for pencils of C faces: slot indices, the C+1
// cells' coefficients W, the contraction results A (NA C F p^(d-1)) and a
// scratch of 5 C F p^(d-1) that overlays W when W is large enough (W is dead
// after the normal contraction).
template <int D, int P, typename T, int PH>
size_t face_lds_bytes(int C)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    constexpr int F = Fld<D, PH>::F;
    const size_t hdr = (((C + 1) * (sizeof(long long) + sizeof(int)) + 15) / 16) * 16;
    const size_t Q = (size_t)C * F * K;
    const size_t W = (size_t)(C + 1) * F * NP;
    const size_t NA = Fld<D, PH>::GRAD ? 4 : 2;
    const size_t tot = W + NA * Q + (W >= 5 * Q ? 0 : 5 * Q);
    return hdr + sizeof(T) * tot;
}

// ---------------------------------------------------------------------------
// volume kernel
// ---------------------------------------------------------------------------

template <int D, int P, typename T, int PH>
__device__ __forceinline__ void vol_body(const Phys &ph, const Geo &geo, const VolArgs &a, unsigned char *smem,
                                         long long tile)
{
    constexpr int NP = ipow(P, D);
    constexpr int K = NP / P;
    constexpr int Fc = Fld<D, PH>::Fc;
    constexpr int F = Fld<D, PH>::F;
    constexpr bool GRAD = Fld<D, PH>::GRAD;
    constexpr int FNP = F * NP;
    const bool forced = a.forcing != nullptr;
    const int Fx = F + (forced ? D : 0);
    const int C = a.cells_per_block;
    const int CNP = C * NP;                   // one field of the tile
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = tile * C;

    // LDS, field-major: X0/X1 [field][cell][point], G [axis][field][cell][point]
    long long *fidx = (long long *)smem;      // [C][D][2] lower/upper face index per axis
    double *cellv = (double *)(fidx + 2 * D * C);   // [C]: wiggle source
    int *blkflag = (int *)(cellv + C);
    T *X0 = (T *)(smem + ((C * (2 * D * sizeof(long long) + sizeof(double)) + sizeof(int) + 15) / 16) * 16);
    T *X1 = X0 + Fx * CNP;
    T *G = X1 + Fx * CNP;
    const Tab<T> &tb = TabSel<T>::get(P);

    // 1. load the tile's weights (and forcing coefficients); per-cell data
    const long long gbase = c0 * FNP, gend = NC * FNP;
    for (int i = tid; i < C * FNP; i += nt) {
        const int c = i / FNP, r = i - c * FNP;
        const int f = r / NP, j = r - f * NP;
        long long gi = gbase + i;
        if (gi >= gend) gi = (NC - 1) * FNP + r;
        X0[f * CNP + c * NP + j] = (T)a.cur[gi];
    }
    if (forced) {
        for (int i = tid; i < C * D * NP; i += nt) {
            const int c = i / (D * NP), r = i - c * (D * NP);
            const int f = r / NP, j = r - f * NP;
            long long cc = c0 + c;
            if (cc >= NC) cc = NC - 1;
            X0[(F + f) * CNP + c * NP + j] = (T)a.forcing[cc * D * NP + r];
        }
    }
    if (tid == 0) *blkflag = 0;
    for (int cl = tid; cl < C; cl += nt) {
        long long cc = c0 + cl;
        if (cc >= NC) cc = NC - 1;
        int co[3];
        long long t = cc;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            co[b] = (int)(t % geo.n[b]);
            t /= geo.n[b];
        }
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const int nfa = geo.nf[ax];
            long long flo = 0, fhi = 0, mul = 1;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int nb = (b == ax) ? nfa : geo.n[b];
                int ilo = co[b], ihi = co[b];
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
        if (PH == 2) {
            // sensor S of the current state and the wiggle source (Sec. 4.1)
            const double *wr = a.cur + cc * FNP;
            double all = 0.0, top = 0.0;
            for (int m = 0; m < NP; ++m) {
                const double x = wr[m];
                all += x * x;
                bool tp = false;
                int r = m;
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    tp = tp || (r % P == P - 1);
                    r /= P;
                }
                if (tp) top += x * x;
            }
            const double Sv = all > 0.0 ? top / all : 0.0;
            const double Rp = a.R_prev ? a.R_prev[cc] : 0.0;
            cellv[cl] = (Sv > ph.s_thr) ? ph.f_w * fmax(0.0, Rp) : 0.0;
        }
    }
    __syncthreads();

    // 2. point values of all fields: one operator pass per axis
    line_pass<P, D, 0, T, M_B, false>(X0, X1, Fx * C);
    __syncthreads();
    line_pass<P, D, 1, T, M_B, false>(X1, X0, Fx * C);
    __syncthreads();
    if (D == 3) {
        line_pass<P, D, (D == 3 ? 2 : 0), T, M_B, false>(X0, X1, Fx * C);
        __syncthreads();
    }
    T *U = (D == 3) ? X1 : X0;
    T *Wk = (D == 3) ? X0 : X1;

    // 3. collocation gradients d/dxi of the stored fields
    if (GRAD) {
        line_pass<P, D, 0, T, M_D, false>(U, G, F * C);
        line_pass<P, D, 1, T, M_D, false>(U, G + F * CNP, F * C);
        if (D == 3) line_pass<P, D, (D == 3 ? 2 : 0), T, M_D, false>(U, G + 2 * F * CNP, F * C);
        __syncthreads();
    }

    // 4. point fluxes (weighted by the volume Gauss weights) and sources
    const T gamma = (T)ph.gamma;
    for (int q = tid; q < CNP; q += nt) {
        const int j = q % NP;                  // q = c * NP + j
        T u[F + D];
#pragma unroll
        for (int f = 0; f < F; ++f) u[f] = U[f * CNP + q];
        if (forced) {
#pragma unroll
            for (int i = 0; i < D; ++i) u[F + i] = U[(F + i) * CNP + q];
        }
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
        if (PH == 2) {
            cs = sqrt(gamma * s.p * s.ir);
            eps = (T)ph.av_scale * clamp_alpha(u[Fc], (T)ph.alpha_max) * cs * (T)ph.eps_fac;
        }
#pragma unroll
        for (int b = 0; b < D; ++b) {
            T fl[D + 2];
            euler_flux<D, T>(u, s, b, fl);
            if (PH == 1 || (PH == 2 && ph.ns_on)) {
                T fv[D + 2];
                ns_flux<D, T>(u, s, g, b, gamma, (T)ph.nu, (T)ph.kappa, fv);
#pragma unroll
                for (int f = 0; f < D + 2; ++f) fl[f] -= fv[f];
            }
            if (PH == 2) {
#pragma unroll
                for (int f = 0; f < D + 2; ++f) fl[f] -= eps * g[b][f];
            }
#pragma unroll
            for (int f = 0; f < D + 2; ++f) G[(b * F + f) * CNP + q] = wq * fl[f];
        }
        // sources, scaled to the common prefactor: Q = (h/2) w_j src
        const T hw = (T)ph.half_h * wq;
        T src[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) src[f] = T(0);
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
        for (int f = 0; f < D + 2; ++f) U[f * CNP + q] = hw * src[f];
        if (PH == 2) {
            T div = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) div += (g[i][1 + i] - s.v[i] * g[i][0]) * s.ir;
            const T asrc = (T)ph.f_v * fmax(T(0), -div) + (T)cellv[q / NP] - u[Fc] * cs * (T)ph.sink;
            U[Fc * CNP + q] = hw * asrc;
        }
    }
    __syncthreads();

    // 5. Q += sum_a D_a^T (w f_a)
    line_pass<P, D, 0, T, M_DT, true>(G, U, Fc * C);
    __syncthreads();
    line_pass<P, D, 1, T, M_DT, true>(G + F * CNP, U, Fc * C);
    __syncthreads();
    if (D == 3) {
        line_pass<P, D, (D == 3 ? 2 : 0), T, M_DT, true>(G + 2 * F * CNP, U, Fc * C);
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
            const long long flo = fidx[(c * D + ax) * 2], fhi = fidx[(c * D + ax) * 2 + 1];
            const T Fl = fb[flo * (Fc * K) + f * K + k];
            const T Fu = fb[fhi * (Fc * K) + f * K + k];
            const int lo = k % S, hi = k / S;
            T *po = U + f * CNP + c * NP + lo + hi * S * P;
#pragma unroll
            for (int i = 0; i < P; ++i) po[i * S] += tb.Lm[i] * Fl - tb.Lp[i] * Fu;
        }
        __syncthreads();
    }

    // 7. point -> modal projection of every stored field
    line_pass<P, D, 0, T, M_BT, false>(U, Wk, F * C);
    __syncthreads();
    line_pass<P, D, 1, T, M_BT, false>(Wk, U, F * C);
    __syncthreads();
    if (D == 3) {
        line_pass<P, D, (D == 3 ? 2 : 0), T, M_BT, false>(U, Wk, F * C);
        __syncthreads();
    }
    const T *V = (D == 3) ? Wk : U;

    // 8. RK combination in FP64 and write-back
    const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
    const double pref = ph.pref;
    int bad = 0;
    for (int i = tid; i < C * FNP; i += nt) {
        const int c = i / FNP, r = i - c * FNP;
        const int f = r / NP, j = r - f * NP;
        const long long gi = gbase + i;
        if (gi >= gend) continue;
        const double L = pref * (double)V[f * CNP + c * NP + j];
        const double cur = a.cur[gi];
        double o = a.c_cur * cur + a.c_L * dt * L;
        if (a.base) o += a.c_base * a.base[gi];
        if (a.out2) {
            double o2 = a.d_cur * cur + a.d_L * dt * L;
            if (a.x2) o2 += a.d_x2 * a.x2[gi];
            a.out2[gi] = o2;
        }
        a.out[gi] = o;
        if (!isfinite(o)) bad |= 2;
    }
    if (bad) atomicOr(blkflag, bad);
    __syncthreads();

    // 9. per-cell checks (mean density and pressure) and, at stage 1, d ln S / dt
    for (int cl = tid; cl < C; cl += nt) {
        const long long cc = c0 + cl;
        if (cc >= NC) continue;
        const double *o = a.out + cc * FNP;
        const double rho = o[0];
        double m2 = 0.0;
        for (int i = 0; i < D; ++i) m2 += o[(1 + i) * NP] * o[(1 + i) * NP];
        const double pm = (ph.gamma - 1.0) * (o[(D + 1) * NP] - 0.5 * m2 / rho);
        if (a.check && !(rho > 0.0 && pm > 0.0)) atomicOr(blkflag, 1);
        if (PH == 2 && a.R_out) {
            const double *wr = a.cur + cc * FNP;
            double Aa = 0.0, Tt = 0.0, ad = 0.0, td = 0.0;
            for (int m = 0; m < NP; ++m) {
                const double x = wr[m];
                const double xd = pref * (double)V[cl * NP + m];
                Aa += x * x;
                ad += x * xd;
                bool tp = false;
                int r = m;
                for (int b = 0; b < D; ++b) {
                    tp = tp || (r % P == P - 1);
                    r /= P;
                }
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

// Grouped volume/stage kernel over every box of one (dim, order) group.
template <int D, int P, typename T, int PH>
__global__ void __launch_bounds__(512) vol_kernel_batched(const BoxDesc *boxes, int nbox, StageDesc sd)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = xcd_block(blockIdx.x, gridDim.x);
    const int i = owner_box(boxes, nbox, b, 0);
    const BoxDesc &B = boxes[i];
    const Phys ph = B.ph;
    const Geo geo = B.geo;
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
    vol_body<D, P, T, PH>(ph, geo, a, smem, b - B.start[0]);
}

template <int D, int P, typename T, int PH>
size_t vol_lds_bytes(int C, int Fx)
{
    constexpr int NP = ipow(P, D);
    constexpr int F = Fld<D, PH>::F;
    const size_t hdr = ((C * (2 * D * sizeof(long long) + sizeof(double)) + sizeof(int) + 15) / 16) * 16;
    return hdr + sizeof(T) * ((size_t)2 * C * Fx * NP + (size_t)C * D * F * NP);
}

// ---------------------------------------------------------------------------
// CFL kernel: maxima of c_s and |v| over the volume Gauss points (eq. timestep)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

template <int D, int P, int PH>
__device__ __forceinline__ void cfl_body(const Phys &ph, const Geo &geo, const CflArgs &a, unsigned char *smem,
                                         long long tile)
{
    constexpr int NP = ipow(P, D);
    constexpr int Fc = D + 2;
    constexpr int FNP = Fld<D, PH>::F * NP;
    const int C = a.cells_per_block;
    const int tid = threadIdx.x, nt = blockDim.x;
    const long long NC = geo.ncells;
    const long long c0 = tile * C;
    double *X0 = (double *)smem;
    double *X1 = X0 + C * Fc * NP;
    double *red = X1 + C * Fc * NP;      // [2][nt]
    for (int i = tid; i < C * Fc * NP; i += nt) {
        const int c = i / (Fc * NP), r = i - c * (Fc * NP);
        long long cc = c0 + c;
        if (cc >= NC) cc = NC - 1;
        X0[i] = a.w[cc * FNP + r];
    }
    __syncthreads();
    axis_pass<P, D, 0, double, M_B, false, Fc>(X0, Fc * NP, X1, Fc * NP, C);
    __syncthreads();
    axis_pass<P, D, 1, double, M_B, false, Fc>(X1, Fc * NP, X0, Fc * NP, C);
    __syncthreads();
    if (D == 3) {
        axis_pass<P, D, (D == 3 ? 2 : 0), double, M_B, false, Fc>(X0, Fc * NP, X1, Fc * NP, C);
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
        cmax = nanmax(cmax, sqrt(ph.gamma * s.p * s.ir));   // NaN propagates into dt
        vmax = nanmax(vmax, sqrt(v2));
    }
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
        a.part[2 * tile] = red[0];
        a.part[2 * tile + 1] = red[nt];
    }
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(512) cfl_kernel(Phys ph, Geo geo, CflArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    cfl_body<D, P, PH>(ph, geo, a, smem, blockIdx.x);
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(512) cfl_kernel_batched(const BoxDesc *boxes, int nbox)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const long long b = blockIdx.x;
    const int i = owner_box(boxes, nbox, b, 2);
    const Phys ph = boxes[i].ph;
    const Geo geo = boxes[i].geo;
    CflArgs a;
    a.w = boxes[i].reg[0];
    a.part = boxes[i].cfl_part;
    a.cells_per_block = boxes[i].cfl_cells;
    cfl_body<D, P, PH>(ph, geo, a, smem, b - boxes[i].start[2]);
}

template <int D, int P>
size_t cfl_lds_bytes(int C, int nt)
{
    constexpr int NP = ipow(P, D);
    return sizeof(double) * ((size_t)2 * C * (D + 2) * NP + 2 * (size_t)nt);
}

}  // namespace dgk
