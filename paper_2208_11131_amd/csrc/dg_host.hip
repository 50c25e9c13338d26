// dg_host.hip -- host runtime of the DG library: C ABI (include/dg.h),
// per-order tables, buffer management, launch configuration and the SSP-RK
// stage sequencing.  Also holds the small reduction kernels (CFL finalise,
// conserved totals).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dg.h"
#include "dg_common.hpp"
#include "dg_tiles.hpp"
#include "dg_registry.hpp"

using dgk::KernelSet;
using dgk::MAXP;
using dgk::Tab;

// ---------------------------------------------------------------------------
// tables (long double on the host, rounded once to FP64 / FP32)
// ---------------------------------------------------------------------------

namespace {

typedef long double LD;

// Unscaled Legendre P_0..P_lmax at x and derivatives, with
// P_{l+1} = ((2l+1) x P_l - l P_{l-1})/(l+1) and P'_{l+1} = (l+1) P_l + x P'_l.
void leg(int lmax, LD x, LD *P, LD *dP)
{
    P[0] = 1.0L;
    dP[0] = 0.0L;
    for (int l = 0; l < lmax; ++l) {
        const LD pm = l > 0 ? P[l - 1] : 0.0L;
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * pm) / (l + 1);
        dP[l + 1] = (l + 1) * P[l] + x * dP[l];
    }
}

// scaled basis Pt_l = sqrt(2l+1) P_l and its derivative
void sleg(int lmax, LD x, LD *P, LD *dP)
{
    leg(lmax, x, P, dP);
    for (int l = 0; l <= lmax; ++l) {
        const LD s = sqrtl(2.0L * l + 1.0L);
        P[l] *= s;
        dP[l] *= s;
    }
}

// n-point Gauss-Legendre nodes (ascending) and weights by Newton iteration.
void gauss_ld(int n, LD *x, LD *w)
{
    LD P[64], dP[64];
    for (int i = 0; i < n; ++i) {
        LD z = cosl(3.14159265358979323846264338327950288L * (4.0L * (n - i) - 1.0L) / (4.0L * n + 2.0L));
        for (int it = 0; it < 60; ++it) {
            leg(n, z, P, dP);
            const LD dz = P[n] / dP[n];
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        leg(n, z, P, dP);
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dP[n] * dP[n]);
    }
}

template <typename T>
void round_tab(const Tab<LD> &s, Tab<T> &d)
{
    for (int i = 0; i < MAXP; ++i) {
        for (int j = 0; j < MAXP; ++j) {
            d.B[i][j] = (T)s.B[i][j];
            d.Bd[i][j] = (T)s.Bd[i][j];
            d.D[i][j] = (T)s.D[i][j];
        }
        d.g[i] = (T)s.g[i];
        d.Lp[i] = (T)s.Lp[i];
        d.Lm[i] = (T)s.Lm[i];
        d.ep[i] = (T)s.ep[i];
        d.em[i] = (T)s.em[i];
        d.rvL[i] = (T)s.rvL[i];
        d.rvR[i] = (T)s.rvR[i];
        d.rdL[i] = (T)s.rdL[i];
        d.rdR[i] = (T)s.rdR[i];
        for (int j = 0; j < MAXP; ++j) {
            d.prvL[i][j] = (T)s.prvL[i][j];
            d.prvR[i][j] = (T)s.prvR[i][j];
            d.prdL[i][j] = (T)s.prdL[i][j];
            d.prdR[i][j] = (T)s.prdR[i][j];
        }
    }
}

// Tables of order P (Sec. 2.3, 2.4, 3.2).
void build_tab(int P, Tab<LD> &t)
{
    memset(&t, 0, sizeof(t));
    LD x[MAXP], w[MAXP], Pv[64], dPv[64];
    gauss_ld(P, x, w);
    for (int j = 0; j < P; ++j) {
        sleg(P - 1, x[j], Pv, dPv);
        for (int l = 0; l < P; ++l) {
            t.B[l][j] = Pv[l];
            t.Bd[l][j] = dPv[l];
        }
        t.g[j] = w[j];
    }
    // barycentric weights -> Lagrange derivative matrix and end values
    LD lam[MAXP];
    for (int j = 0; j < P; ++j) {
        LD pr = 1.0L;
        for (int k = 0; k < P; ++k)
            if (k != j) pr *= (x[j] - x[k]);
        lam[j] = 1.0L / pr;
    }
    for (int j = 0; j < P; ++j) {
        LD diag = 0.0L;
        for (int k = 0; k < P; ++k) {
            if (k == j) continue;
            const LD v = (lam[k] / lam[j]) / (x[j] - x[k]);
            t.D[j][k] = v;
            diag -= v;
        }
        t.D[j][j] = diag;
        LD lp = 1.0L, lm = 1.0L;
        for (int k = 0; k < P; ++k) {
            if (k == j) continue;
            lp *= (1.0L - x[k]) / (x[j] - x[k]);
            lm *= (-1.0L - x[k]) / (x[j] - x[k]);
        }
        t.Lp[j] = lp;
        t.Lm[j] = lm;
    }
    for (int m = 0; m < P; ++m) {
        t.ep[m] = sqrtl(2.0L * m + 1.0L);
        t.em[m] = (m & 1 ? -1.0L : 1.0L) * sqrtl(2.0L * m + 1.0L);
    }
    // Recovery (Sec. 3.2): projection of the two sides onto the normal
    // Legendre polynomials of degree 0..n+1 on K* (xi* in [-1,1], overlap f),
    //   A_side(la, m) = (1/2) int_half Pt_la(xi*) Pt_m(2 f xi* +- 1) dxi*,
    // then value / xi*-derivative of the recovered expansion at xi* = 0.
    const LD f = (P - 1) <= 2 ? 0.75L : 1.0L;
    LD xq[24], wq[24], P0[64], dP0[64];
    gauss_ld(20, xq, wq);
    sleg(P, 0.0L, P0, dP0);
    LD AL[MAXP + 1][MAXP], AR[MAXP + 1][MAXP];
    for (int m = 0; m < P; ++m)
        for (int la = 0; la <= P; ++la) {
            LD sl = 0, sr = 0;
            for (int q = 0; q < 20; ++q) {
                LD a[64], da[64], b[64], db[64];
                const LD xsL = 0.5L * (xq[q] - 1.0L);   // [-1, 0]
                const LD xsR = 0.5L * (xq[q] + 1.0L);   // [0, 1]
                sleg(P, xsL, a, da);
                sleg(P - 1, 2.0L * f * xsL + 1.0L, b, db);
                sl += 0.5L * wq[q] * 0.5L * a[la] * b[m];
                sleg(P, xsR, a, da);
                sleg(P - 1, 2.0L * f * xsR - 1.0L, b, db);
                sr += 0.5L * wq[q] * 0.5L * a[la] * b[m];
            }
            AL[la][m] = sl;
            AR[la][m] = sr;
        }
    // recovered expansion truncated at normal degree lmax: value and
    // xi*-derivative at the face of the sides' contributions
    auto vectors = [&](int lmax, int m, LD *vl, LD *vr, LD *dl, LD *dr) {
        *vl = *vr = *dl = *dr = 0;
        for (int la = 0; la <= lmax; ++la) {
            *vl += AL[la][m] * P0[la];
            *vr += AR[la][m] * P0[la];
            *dl += AL[la][m] * dP0[la];
            *dr += AR[la][m] * dP0[la];
        }
    };
    for (int m = 0; m < P; ++m) vectors(P, m, &t.rvL[m], &t.rvR[m], &t.rdL[m], &t.rdR[m]);
    // total-degree basis: transverse degree tau leaves normal degrees
    // m <= n - tau, recovered to n + 1 - tau
    for (int tau = 0; tau < P; ++tau)
        for (int m = 0; m + tau < P; ++m)
            vectors(P - tau, m, &t.prvL[tau][m], &t.prvR[tau][m], &t.prdL[tau][m], &t.prdR[tau][m]);
}

struct Tables {
    Tab<double> d[MAXP + 1];
    Tab<float> f[MAXP + 1];
};

Tables *g_tables = nullptr;
std::mutex g_mu;
unsigned long long g_uploaded = 0;   // bit mask of devices with tables

dg_status ensure_tables(int dev)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tables) {
        Tables *t = new (std::nothrow) Tables;
        if (!t) return DG_ENOMEM;
        memset(t, 0, sizeof(*t));
        for (int P = 1; P <= MAXP; ++P) {
            Tab<LD> s;
            build_tab(P, s);
            round_tab(s, t->d[P]);
            round_tab(s, t->f[P]);
        }
        g_tables = t;
    }
    if (dev < 64 && (g_uploaded >> dev) & 1ULL) return DG_OK;
    if (dgk::dgk_upload_2d_f64(g_tables->d, g_tables->f) || dgk::dgk_upload_3d_f64(g_tables->d, g_tables->f) ||
        dgk::dgk_upload_2d_f32(g_tables->d, g_tables->f) || dgk::dgk_upload_3d_f32(g_tables->d, g_tables->f))
        return DG_EDEVICE;
    if (dev < 64) g_uploaded |= 1ULL << dev;
    return DG_OK;
}

dg_status ensure_scratch(int dev);

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ double nanmax2(double a, double b) { return (b > a || b != b) ? b : a; }

// Maxima of the (c_s, |v|) pairs part[0 .. nblk) with one block of
// kFinT threads: each pair is one 16-byte load, four independent
// accumulators per thread keep four loads in flight, then a tree in LDS.
// Max is order independent, so the result does not depend on the split.
constexpr int kFinT = 1024;

__device__ __forceinline__ void cfl_reduce_pairs(const double *part, long long nblk, double *cm, double *vm)
{
    __shared__ double rc[kFinT], rv[kFinT];
    const int t = threadIdx.x;
    const double2 *pp = (const double2 *)part;
    double c[4] = {0.0, 0.0, 0.0, 0.0}, v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long b0 = t; b0 < nblk; b0 += 4 * kFinT) {
        double2 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long b = b0 + (long long)u * kFinT;
            x[u] = b < nblk ? pp[b] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = nanmax2(c[u], x[u].x);
            v[u] = nanmax2(v[u], x[u].y);
        }
    }
    rc[t] = nanmax2(nanmax2(c[0], c[1]), nanmax2(c[2], c[3]));
    rv[t] = nanmax2(nanmax2(v[0], v[1]), nanmax2(v[2], v[3]));
    __syncthreads();
    for (int st = kFinT / 2; st > 0; st >>= 1) {
        if (t < st) {
            rc[t] = nanmax2(rc[t], rc[t + st]);
            rv[t] = nanmax2(rv[t], rv[t + st]);
        }
        __syncthreads();
    }
    *cm = rc[0];
    *vm = rv[0];
}

// dt = f_CFL h / (2 p (c_max + v_max)) from the CFL kernel's partial maxima.
__global__ void __launch_bounds__(kFinT) cfl_finalize(const double *part, int nblk, double *res, double *dt_copy,
                                                      double num)
{
    double cm, vm;
    cfl_reduce_pairs(part, nblk, &cm, &vm);
    if (threadIdx.x == 0) {
        const double dt = num / (cm + vm);
        res[0] = dt;
        res[1] = cm;
        res[2] = vm;
        if (dt_copy) dt_copy[0] = dt;
    }
}

// Per-box CFL reduction of a grouped launch: block i reduces box i's partials.
__global__ void __launch_bounds__(kFinT) cfl_finalize_batched(const dgk::BoxDesc *boxes, double cfl)
{
    const dgk::BoxDesc &B = boxes[blockIdx.x];
    double cm, vm;
    cfl_reduce_pairs(B.cfl_part, B.nblocks[2], &cm, &vm);
    if (threadIdx.x == 0) {
        const double num = cfl * B.ph.h / (2.0 * B.ph.order);
        B.dt[0] = num / (cm + vm);
        B.dt[1] = cm;
        B.dt[2] = vm;
    }
}

// Caller-given step sizes of a batched step (dg_batch_step_dt): box i of a
// grouped launch takes dt_in[bidx] as its dt (read when the step runs).
__global__ void __launch_bounds__(64) dt_in_batched(const dgk::BoxDesc *boxes, int n, const double *dt_in)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) boxes[i].dt[0] = dt_in[boxes[i].bidx];
}

// The same for one box: dst[0] = src[0].
__global__ void __launch_bounds__(64) dt_in_single(const double *src, double *dst)
{
    if (threadIdx.x == 0) dst[0] = src[0];
}

// Neumaier-compensated add of x into (s, c).
__device__ __forceinline__ void nadd(double &s, double &c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// Per-block compensated partial sums of |K| w_0 over a contiguous cell range
// (fixed thread/cell assignment and combination order: deterministic).
__global__ void totals_partial(const double *w, long long NC, int F, int NP, int Fc, double vol, int chunk,
                               double *part)
{
    __shared__ double ss[256 * 6], cc[256 * 6];   // up to 6 conserved fields
    const long long c0 = (long long)blockIdx.x * chunk;
    const int tid = threadIdx.x;
    for (int f = 0; f < Fc; ++f) {
        double s = 0.0, c = 0.0;
        for (long long k = c0 + tid; k < c0 + chunk && k < NC; k += blockDim.x)
            nadd(s, c, vol * w[(k * F + f) * (long long)NP]);
        ss[f * 256 + tid] = s;
        cc[f * 256 + tid] = c;
    }
    __syncthreads();
    if (tid < Fc) {
        double s = 0.0, c = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            nadd(s, c, ss[tid * 256 + t]);
            c += cc[tid * 256 + t];
        }
        part[(blockIdx.x * Fc + tid) * 2] = s;
        part[(blockIdx.x * Fc + tid) * 2 + 1] = c;
    }
}

__global__ void totals_final(const double *part, int nblk, int Fc, double *out)
{
    const int f = threadIdx.x;
    if (f < Fc) {
        double s = 0.0, c = 0.0;
        for (int b = 0; b < nblk; ++b) {
            nadd(s, c, part[(b * Fc + f) * 2]);
            c += part[(b * Fc + f) * 2 + 1];
        }
        out[f] = s + c;
    }
}

int roundup(int x, int m) { return (x + m - 1) / m * m; }

using dgk::TileEntry;

// Tuned tiles for this (dim, order, precision, physics, forcing), if any.
const TileEntry *find_tiles(int dim, int order, int prec, int phys, int forced)
{
    for (size_t i = 0; i < dgk::kNumTiles; ++i) {
        const TileEntry &t = dgk::kTiles[i];
        if (t.dim == dim && t.order == order && t.prec == prec && t.phys == phys && t.forced == forced) return &t;
    }
    return nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

struct dg_ctx {
    int dim, P, F, Fc, NP, K;
    int NM;      // stored modes per field: NP (tensor basis) or the total-degree count
    long long ncells;
    dgk::Phys ph;
    dgk::Geo geo;
    int precision;
    double cfl;
    int device;
    bool grad;
    int phys;    // 0 Euler, 1 Navier-Stokes, 2 artificial viscosity, 3 Navier-Stokes + tracer,
                 // 4..7 the same four on the total-degree basis
    KernelSet ks, ks64;
    const void *vol_fixed[2];   // fixed-tile volume kernels (no forcing / forcing) for the tile in use, or null
    const void *face_fixed;     // fixed-tile face kernel for the tile in use, or null
    bool fin_pending;           // the next face launch carries the CFL finalize
    double *fin_dt_copy;        // its optional second copy of dt
    int vol_C, vol_T, face_C, face_T, cfl_C, cfl_T;
    int cfl_tiles;                 // tiles of cfl_C cells (one block each in a grouped launch)
    int cfl_blocks;                // blocks (= partials) of a single-box CFL launch, at most kCflBlocks
    size_t vol_lds, vol_lds_forced, face_lds, cfl_lds;
    int stages;
    int limiter;                   // positivity limiter after every stage (Sec. 4.2)
    int lim_C, lim_T;
    size_t lim_lds;
    double *reg[3];
    void *fb;
    size_t fb_bytes;
    double *R[2];
    int rpar;
    double *cfl_part;              // [cfl_tiles][2]
    double *scal;                  // [0] dt, [1] cmax, [2] vmax, [3..] totals
    int *flag;
    double *tot_part;
    int tot_blocks, tot_chunk;
    const void *forcing;           // driving field at the Gauss points (spts) while forcing is on, else null
    const double *forcing_src;     // the caller's coefficients, converted before the next RHS
    void *spts;                    // [cell][dim][p^d] of the bulk type
    bool forcing_dirty;
    // kernel timing
    int timing;
    std::vector<hipEvent_t> *ev_pool;
    std::vector<int> *ev_kind;     // per recorded pair: 0 face, 1 vol, 2 cfl
    long long ev_used, ev_dropped;
};

namespace {

bool ok(hipError_t e) { return e == hipSuccess; }

void free_bufs(dg_ctx *c)
{
    for (int i = 0; i < 3; ++i)
        if (c->reg[i]) (void)hipFree(c->reg[i]);
    if (c->fb) (void)hipFree(c->fb);
    for (int i = 0; i < 2; ++i)
        if (c->R[i]) (void)hipFree(c->R[i]);
    if (c->cfl_part) (void)hipFree(c->cfl_part);
    if (c->scal) (void)hipFree(c->scal);
    if (c->flag) (void)hipFree(c->flag);
    if (c->tot_part) (void)hipFree(c->tot_part);
    if (c->spts) (void)hipFree(c->spts);
}

void get_kernels(int dim, int prec, int P, int phys, KernelSet *k)
{
    if (dim == 2)
        (prec == DG_PREC_FP64 ? dgk::dgk_get_2d_f64 : dgk::dgk_get_2d_f32)(P, phys, k);
    else
        (prec == DG_PREC_FP64 ? dgk::dgk_get_3d_f64 : dgk::dgk_get_3d_f32)(P, phys, k);
}

// Fixed-tile volume kernel of the tuned table for this tile, if one was built.
const void *get_vol_fixed(int dim, int prec, int P, int phys, int C, int NT, int forced, int batched = 0)
{
    if (dim == 2)
        return (prec == DG_PREC_FP64 ? dgk::dgk_vol_fixed_2d_f64 : dgk::dgk_vol_fixed_2d_f32)(P, phys, C, NT, forced,
                                                                                              batched);
    return (prec == DG_PREC_FP64 ? dgk::dgk_vol_fixed_3d_f64 : dgk::dgk_vol_fixed_3d_f32)(P, phys, C, NT, forced,
                                                                                          batched);
}

// Fixed-tile face kernel of the tuned table for this tile, if one was built.
const void *get_face_fixed(int dim, int prec, int P, int phys, int C, int NT, int batched = 0)
{
    if (dim == 2)
        return (prec == DG_PREC_FP64 ? dgk::dgk_face_fixed_2d_f64 : dgk::dgk_face_fixed_2d_f32)(P, phys, C, NT,
                                                                                                batched);
    return (prec == DG_PREC_FP64 ? dgk::dgk_face_fixed_3d_f64 : dgk::dgk_face_fixed_3d_f32)(P, phys, C, NT, batched);
}

constexpr size_t LDS_MAX = 160 * 1024;

// Allow `bytes` of dynamic LDS for kernel fn.  A failure is returned and
// cleared from the runtime's error state (nothing stale is left for the
// caller's next HIP call to report).
bool set_lds(const void *fn, size_t bytes)
{
    if (!fn) return false;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// Blocks of a single-box CFL launch (each loops over tiles): bounds the
// partial maxima the finalize reads, whatever the mesh size.
constexpr int kCflBlocks = 4096;

}  // namespace

// Static scratch of the allocation-free entry point dg_max_dt_noalloc: the
// CFL kernel's per-block (c_s, |v|) maxima, kScratchDoubles doubles (64 KiB).
// Each device holds its own copy until the process ends.  In host code the
// name stands for a host-side handle, not a device address: host code uses
// g_scratch_dev[device] (from hipGetSymbolAddress at dg_init) instead.
constexpr int kScratchDoubles = 2 * kCflBlocks;
__device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), taken once
// per device at context creation.
dg_status ensure_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return DG_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch_dev[dev]) return DG_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return DG_EDEVICE;
    }
    g_scratch_dev[dev] = (double *)p;
    return DG_OK;
}

constexpr long long EV_MAX = 16384;

// Launch a kernel; with timing on, bracket it by a pair of events.
dg_status launch(dg_ctx *c, int kind, const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                 hipStream_t s)
{
    if (grid.x == 0) return DG_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c && c->timing) {
        if (c->ev_used < EV_MAX) {
            const size_t need = 2 * (size_t)(c->ev_used + 1);
            while (c->ev_pool->size() < need) {
                hipEvent_t e;
                // timing-only events: no system-scope fence (no cache writeback /
                // invalidation between the kernels being measured)
                if (!ok(hipEventCreateWithFlags(&e, hipEventDisableSystemFence))) return DG_EDEVICE;
                c->ev_pool->push_back(e);
            }
            e0 = (*c->ev_pool)[2 * c->ev_used];
            e1 = (*c->ev_pool)[2 * c->ev_used + 1];
            c->ev_kind->push_back(kind > 2 ? 2 : kind);
            ++c->ev_used;
            if (!ok(hipEventRecord(e0, s))) return DG_EDEVICE;
        } else {
            ++c->ev_dropped;
        }
    }
    if (!ok(hipLaunchKernel(fn, grid, block, args, lds, s))) return DG_EDEVICE;
    if (e1 && !ok(hipEventRecord(e1, s))) return DG_EDEVICE;
    return DG_OK;
}

// Gauss-point values of the caller's driving-field coefficients, after a
// dg_set_forcing (enqueued on the stream of the next RHS).
dg_status convert_forcing(dg_ctx *c, hipStream_t s)
{
    const int FA = c->NP >= 256 ? 1 : 256 / c->NP;
    long long narr = c->ncells * c->dim;
    const double *src = c->forcing_src;
    void *dst = c->spts;
    void *args[] = {&src, &dst, &narr};
    const long long groups = (narr + FA - 1) / FA;
    const dim3 g((unsigned)std::min<long long>(groups, 1LL << 20));   // grid-stride kernel
    if (!ok(hipLaunchKernel(c->ks.fpts, g, dim3(256), args, 0, s))) return DG_EDEVICE;
    c->forcing_dirty = false;
    return DG_OK;
}

// One RHS evaluation of `in` followed by the stage combination of VolArgs.
dg_status stage(dg_ctx *c, dgk::VolArgs va, hipStream_t s)
{
    if (c->forcing && c->forcing_dirty) {
        const dg_status fs = convert_forcing(c, s);
        if (fs != DG_OK) return fs;
    }
    dgk::FaceArgs fa;
    fa.w = va.cur;
    fa.fb = c->fb;
    fa.faces_per_block = c->face_C;
    fa.cfl_part = nullptr;
    fa.cfl_res = nullptr;
    fa.cfl_dt_copy = nullptr;
    fa.cfl_num = 0.0;
    fa.cfl_nblk = 0;
    if (c->fin_pending) {      // the CFL finalize of this step rides on this launch
        fa.cfl_part = c->cfl_part;
        fa.cfl_res = c->scal;
        fa.cfl_dt_copy = c->fin_dt_copy;
        fa.cfl_num = c->cfl * c->ph.h / (2.0 * c->P);
        fa.cfl_nblk = c->cfl_blocks;
        c->fin_pending = false;
    }
    void *fargs[] = {&c->ph, &c->geo, &fa};
    long long fgx, fgy, fgz;
    dgk::face_grid(c->geo, c->dim, c->face_C, fgx, fgy, fgz);
    dim3 fg((unsigned)fgx, (unsigned)fgy, (unsigned)fgz);
    dg_status st = launch(c, 0, c->face_fixed ? c->face_fixed : c->ks.face, fg, dim3(c->face_T), fargs,
                          c->face_lds, s);
    if (st != DG_OK) return st;
    va.fb = c->fb;
    va.forcing = c->forcing;
    va.flag = c->flag;
    va.cells_per_block = c->vol_C;
    void *vargs[] = {&c->ph, &c->geo, &va};
    dim3 vg((unsigned)((c->ncells + c->vol_C - 1) / c->vol_C));
    const void *vf = c->vol_fixed[c->forcing ? 1 : 0];
    return launch(c, 1, vf ? vf : c->ks.vol, vg, dim3(c->vol_T), vargs, c->forcing ? c->vol_lds_forced : c->vol_lds,
                  s);
}

dgk::VolArgs blank_args()
{
    dgk::VolArgs v;
    memset(&v, 0, sizeof(v));
    return v;
}

// CFL reduction of w.  finalize_now: also launch the one-block finalize (dt in
// c->scal on return to the stream); otherwise the finalize is carried by the
// next face launch of this context (the first stage of the step).
dg_status run_cfl(dg_ctx *c, const double *w, double *dt_copy, hipStream_t s, bool finalize_now = true)
{
    dgk::CflArgs ca;
    ca.w = w;
    ca.part = c->cfl_part;
    ca.cells_per_block = c->cfl_C;
    void *args[] = {&c->ph, &c->geo, &ca};
    dim3 g((unsigned)c->cfl_blocks);
    dg_status st = launch(c, 2, c->ks64.cfl, g, dim3(c->cfl_T), args, c->cfl_lds, s);
    if (st != DG_OK) return st;
    if (!finalize_now) {
        c->fin_pending = true;
        c->fin_dt_copy = dt_copy;
        return DG_OK;
    }
    double num = c->cfl * c->ph.h / (2.0 * c->P);
    const double *part = c->cfl_part;
    int nblk = c->cfl_blocks;
    double *res = c->scal;
    void *fargs[] = {&part, &nblk, &res, &dt_copy, &num};
    return launch(c, 3, (const void *)&cfl_finalize, dim3(1), dim3(kFinT), fargs, 0, s);
}

// Positivity limiter (Sec. 4.2) on the state w, in place.
dg_status run_limiter(dg_ctx *c, double *w, hipStream_t s)
{
    void *args[] = {&c->ph, &c->geo, &w, &c->lim_C};
    dim3 g((unsigned)((c->ncells + c->lim_C - 1) / c->lim_C));
    return launch(c, 4, c->ks64.limit, g, dim3(c->lim_T), args, c->lim_lds, s);
}

// SSP-RK step in Shu-Osher form; dt from the host value or a device pointer.
// With the limiter on, every state a stage writes is limited (the partial sum
// of the fourth 5-stage stage is not a state and is not limited).
dg_status rk_step(dg_ctx *c, double *w, double dt, const double *dt_dev, hipStream_t s)
{
    double *r1 = c->reg[0], *r2 = c->reg[1], *r3 = c->reg[2];
    const double *Rp = c->ph.av_on ? c->R[c->rpar] : nullptr;
    double *Rn = c->ph.av_on ? c->R[c->rpar ^ 1] : nullptr;
    auto A = [&](const double *cur, const double *base, double *out, double cb, double cc, double cl) {
        dgk::VolArgs v = blank_args();
        v.cur = cur;
        v.base = base;
        v.out = out;
        v.c_base = cb;
        v.c_cur = cc;
        v.c_L = cl;
        v.dt = dt;
        v.dt_ptr = dt_dev;
        v.R_prev = Rp;
        v.check = 1;
        return v;
    };
    auto lstage = [&](const dgk::VolArgs &v, hipStream_t st_) {
        dg_status r = stage(c, v, st_);
        if (r == DG_OK && c->limiter) r = run_limiter(c, v.out, st_);
        return r;
    };
    dg_status st = DG_OK;
    switch (c->stages) {
    case 1: {
        dgk::VolArgs v = A(w, nullptr, w, 0.0, 1.0, 1.0);
        v.R_out = Rn;
        st = lstage(v, s);
        break;
    }
    case 2: {
        dgk::VolArgs v = A(w, nullptr, r1, 0.0, 1.0, 1.0);
        v.R_out = Rn;
        if ((st = lstage(v, s)) != DG_OK) break;
        st = lstage(A(r1, w, w, 0.5, 0.5, 0.5), s);
        break;
    }
    case 3: {
        dgk::VolArgs v = A(w, nullptr, r1, 0.0, 1.0, 1.0);
        v.R_out = Rn;
        if ((st = lstage(v, s)) != DG_OK) break;
        if ((st = lstage(A(r1, w, r2, 0.75, 0.25, 0.25), s)) != DG_OK) break;
        st = lstage(A(r2, w, w, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0), s);
        break;
    }
    default: {
        // SSPRK(5,4), Spiteri & Ruuth (2002), Shu-Osher coefficients
        dgk::VolArgs v = A(w, nullptr, r1, 0.0, 1.0, 0.391752226571890);
        v.R_out = Rn;
        if ((st = lstage(v, s)) != DG_OK) break;
        if ((st = lstage(A(r1, w, r2, 0.444370493651235, 0.555629506348765, 0.368410593050371), s)) != DG_OK)
            break;
        if ((st = lstage(A(r2, w, r3, 0.620101851488403, 0.379898148511597, 0.251891774271694), s)) != DG_OK)
            break;
        // u4 -> r1 and the partial sum of the last stage -> w
        v = A(r3, w, r1, 0.178079954393132, 0.821920045606868, 0.544974750228521);
        v.out2 = w;
        v.x2 = r2;
        v.d_x2 = 0.517231671970585;
        v.d_cur = 0.096059710526147;
        v.d_L = 0.063692468666290;
        if ((st = lstage(v, s)) != DG_OK) break;
        st = lstage(A(r1, w, w, 1.0, 0.386708617503269, 0.226007483236906), s);
        break;
    }
    }
    if (st == DG_OK && c->ph.av_on) c->rpar ^= 1;
    return st;
}

}  // namespace

extern "C" {

void dg_av_defaults(dg_av_params *av)
{
    if (!av) return;
    av->enabled = 1;
    av->scale = 1.0;
    av->f_v = 2.5;
    av->f_tau = 0.5;
    av->f_w = 0.2;
    av->s_onset = 1e-4;
    av->alpha_max = 1.0;
}

void dg_options_defaults(dg_options *opt)
{
    if (!opt) return;
    opt->precision = DG_PREC_FP64;
    opt->basis = 0;
    opt->cfl = 0.5;
    opt->cells_per_block = 0;
    opt->faces_per_block = 0;
    opt->vol_threads = 0;
    opt->face_threads = 0;
    opt->limiter = 0;
    opt->tracer = 0;
    opt->tracer_eta = 0.0;
}

const char *dg_status_str(dg_status s)
{
    switch (s) {
    case DG_OK: return "ok";
    case DG_EINVAL: return "invalid argument";
    case DG_ENOMEM: return "out of device memory";
    case DG_EDEVICE: return "HIP device or launch error";
    case DG_ENONPHYSICAL: return "non-positive cell-mean density or pressure";
    case DG_ENONFINITE: return "non-finite weight";
    case DG_EUNSUPPORTED: return "unsupported configuration";
    case DG_ESCRATCH: return "request exceeds the static scratch of the allocation-free entry point";
    }
    return "unknown status";
}

// Cell and face indices are 32-bit inside the kernels (coordinates are
// recovered with 32-bit divisions): every axis product of (n[a] + 1) must
// stay below 2^31.
static const long long kMaxIndex = 2147483647LL;

dg_status dg_init(const dg_mesh *mesh, int order, double gamma, double nu, double kappa, const dg_av_params *av,
                  const dg_options *opt, dg_ctx **out)
{
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!mesh || (mesh->dim != 2 && mesh->dim != 3) || order < 1 || order > MAXP) return DG_EINVAL;
    if (!(gamma > 1.0) || !(nu >= 0.0) || !(kappa >= 0.0) || !std::isfinite(nu) || !std::isfinite(kappa))
        return DG_EINVAL;
    dg_options o;
    dg_options_defaults(&o);
    if (opt) o = *opt;
    if (o.precision != DG_PREC_FP64 && o.precision != DG_PREC_FP32_BULK) return DG_EINVAL;
    if (o.tracer && (!(o.tracer_eta >= 0.0) || !std::isfinite(o.tracer_eta))) return DG_EINVAL;
    if (o.basis != 0 && o.basis != 1) return DG_EINVAL;
    if (!(o.cfl > 0.0) || o.cells_per_block < 0 || o.faces_per_block < 0) return DG_EINVAL;
    if (o.vol_threads < 0 || o.vol_threads > 512 || o.vol_threads % 64 || o.face_threads < 0 ||
        o.face_threads > 512 || o.face_threads % 64)
        return DG_EINVAL;
    const int d = mesh->dim;
    double h = 0.0;
    long long cells = 1;
    for (int a = 0; a < d; ++a) {
        if (mesh->n[a] < 1 || !(mesh->hi[a] > mesh->lo[a])) return DG_EINVAL;
        cells *= (long long)mesh->n[a] + 1;     // bounds the face counts too
        if (cells > kMaxIndex) return DG_EINVAL;
        if (mesh->bc[a] != DG_BC_PERIODIC && mesh->bc[a] != DG_BC_OUTFLOW && mesh->bc[a] != DG_BC_WALL)
            return DG_EINVAL;
        const double ha = (mesh->hi[a] - mesh->lo[a]) / mesh->n[a];
        if (a == 0)
            h = ha;
        else if (fabs(ha - h) > 1e-12 * h)
            return DG_EINVAL;
    }
    const bool av_on = av && av->enabled;
    if (av_on && o.tracer) return DG_EUNSUPPORTED;   // no AV variant carries the tracer
    if (av_on && (!(av->f_tau > 0.0) || !(av->alpha_max >= 0.0) || !(av->scale >= 0.0) || !(av->f_v >= 0.0) ||
                  !(av->f_w >= 0.0) || !(av->s_onset >= 0.0)))
        return DG_EINVAL;

    int dev = 0;
    if (!ok(hipGetDevice(&dev))) return DG_EDEVICE;
    dg_status st = ensure_tables(dev);
    if (st == DG_OK) st = ensure_scratch(dev);
    if (st != DG_OK) return st;

    dg_ctx *c = new (std::nothrow) dg_ctx;
    if (!c) return DG_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->dim = d;
    c->P = order;
    c->Fc = d + 2 + (o.tracer ? 1 : 0);
    c->F = c->Fc + (av_on ? 1 : 0);
    c->NP = 1;
    for (int a = 0; a < d; ++a) c->NP *= order;
    c->K = c->NP / order;
    c->NM = o.basis == 0 ? c->NP : (d == 2 ? order * (order + 1) / 2 : order * (order + 1) * (order + 2) / 6);
    c->device = dev;
    c->precision = o.precision;
    c->cfl = o.cfl;
    c->stages = order == 1 ? 1 : order == 2 ? 2 : order == 3 ? 3 : 5;

    dgk::Geo &g = c->geo;
    c->ncells = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = a < d ? mesh->n[a] : 1;
        g.bc[a] = a < d ? mesh->bc[a] : 0;
        g.nf[a] = g.n[a] + (g.bc[a] != DG_BC_PERIODIC ? 1 : 0);
        c->ncells *= g.n[a];
    }
    g.ncells = c->ncells;
    long long off = 0;
    for (int a = 0; a < 3; ++a) {
        long long nfc = 0;
        if (a < d) {
            nfc = 1;
            for (int b = 0; b < 3; ++b) nfc *= (b == a) ? g.nf[b] : g.n[b];
        }
        g.nfaces[a] = nfc;
        g.fb_off[a] = off;
        off += nfc * c->Fc * c->K;
    }
    const size_t tsz = c->precision == DG_PREC_FP64 ? sizeof(double) : sizeof(float);
    c->fb_bytes = (size_t)off * tsz;

    dgk::Phys &ph = c->ph;
    ph.order = order;
    ph.gamma = gamma;
    ph.nu = nu;
    ph.kappa = kappa;
    ph.h = h;
    ph.two_over_h = 2.0 / h;
    const double fr = (order - 1) <= 2 ? 0.75 : 1.0;
    ph.inv_fh = 1.0 / (fr * h);
    ph.pref = std::pow(2.0, 1 - d) / h;
    ph.half_h = 0.5 * h;
    ph.eta = o.tracer ? o.tracer_eta : 0.0;
    ph.ns_on = (nu > 0.0 || kappa > 0.0 || ph.eta > 0.0) ? 1 : 0;
    ph.av_on = av_on ? 1 : 0;
    if (av_on) {
        ph.av_scale = av->scale;
        ph.f_v = av->f_v;
        ph.sink = order / (av->f_tau * h);
        ph.f_w = av->f_w;
        ph.s_thr = av->s_onset / ((double)order * order);
        ph.alpha_max = av->alpha_max;
        ph.eps_fac = h / order;
    }
    c->grad = ph.ns_on || ph.av_on;
    c->phys = ph.av_on ? 2 : (o.tracer ? 3 : (ph.ns_on ? 1 : 0));
    if (o.basis == 1) c->phys += 4;   // the same physics on the total-degree basis
    get_kernels(d, c->precision, order, c->phys, &c->ks);
    get_kernels(d, DG_PREC_FP64, order, c->phys, &c->ks64);
    if (!c->ks.vol || !c->ks.face || !c->ks64.cfl) {
        delete c;
        return DG_EUNSUPPORTED;
    }

    // launch tiles: explicit options, else the tuned table, else about 256
    // volume points / 128 face points per block
    const TileEntry *te = find_tiles(d, order, c->precision, c->phys, 0);
    if (o.cells_per_block > 0)
        c->vol_C = o.cells_per_block;
    else if (te)
        c->vol_C = te->vol_C;
    else
        c->vol_C = std::max(1, 256 / c->NP);
    while (c->vol_C > 1 && c->ks.vol_lds(c->vol_C, c->F) > LDS_MAX) --c->vol_C;
    if (o.vol_threads > 0)
        c->vol_T = o.vol_threads;
    else if (te && o.cells_per_block == 0)
        c->vol_T = te->vol_T;
    else
        c->vol_T = std::min(512, std::max(64, roundup(c->vol_C * c->NP, 64)));
    // one volume block per vol_C cells: the launch must stay below 2^32 work-items
    if ((c->ncells + c->vol_C - 1) / c->vol_C * (long long)c->vol_T > 0xFFFFFFFFLL) {
        delete c;
        return DG_EUNSUPPORTED;
    }
    c->vol_lds = c->ks.vol_lds(c->vol_C, c->F);
    c->vol_lds_forced = c->ks.vol_lds(c->vol_C, c->F);   // the driving field takes no LDS
    if (c->vol_lds > LDS_MAX) {
        delete c;
        return DG_EUNSUPPORTED;
    }
    if (o.faces_per_block > 0)
        c->face_C = o.faces_per_block;
    else if (te)
        c->face_C = te->face_C;
    else
        c->face_C = std::max(1, 128 / c->K);
    while (c->face_C > 1 && c->ks.face_lds(c->face_C) > 64 * 1024) --c->face_C;
    if (o.face_threads > 0)
        c->face_T = o.face_threads;
    else if (te && o.faces_per_block == 0)
        c->face_T = te->face_T;
    else
        c->face_T = std::min(512, std::max(64, roundup(c->face_C * c->K, 64)));
    c->face_lds = std::max<size_t>(c->ks.face_lds(c->face_C), 256);   // >= the CFL finalize's 16 doubles
    {
        // the face launch (face_grid) within the grid limits and 32-bit block indices
        long long gx, gy, gz;
        dgk::face_grid(c->geo, d, c->face_C, gx, gy, gz);
        if (gx * c->face_T > 0xFFFFFFFFLL || gy > 65535 || gz > 65535 || gx * gy * gz > 0xFFFFFFFFLL) {
            delete c;
            return DG_EUNSUPPORTED;
        }
    }
    // cells per CFL tile: the HBM pass (one item per field and line of the
    // conserved fields) fills one round of the 256 threads
    c->cfl_C = std::max(1, 256 / ((d + 2) * (c->NP / c->P)));
    c->cfl_T = 256;
    while (c->cfl_C > 1 && c->ks64.cfl_lds(c->cfl_C, c->cfl_T) > 64 * 1024) --c->cfl_C;
    c->cfl_lds = c->ks64.cfl_lds(c->cfl_C, c->cfl_T);
    c->limiter = o.limiter ? 1 : 0;
    if (c->limiter) {
        if (!c->ks64.limit) {
            delete c;
            return DG_EUNSUPPORTED;
        }
        // about 64 KiB of LDS per block: two extended-grid arrays per cell
        size_t per_cell = c->ks64.limit_lds(1, 256) - c->ks64.limit_lds(0, 256);
        c->lim_C = (int)std::max<size_t>(1, (64 * 1024) / std::max<size_t>(per_cell, 1));
        if (c->lim_C > 256) c->lim_C = 256;
        if (c->lim_C > c->ncells) c->lim_C = (int)c->ncells;
        c->lim_T = 256;
        c->lim_lds = c->ks64.limit_lds(c->lim_C, c->lim_T);
        if (c->lim_lds > LDS_MAX) {
            delete c;
            return DG_EUNSUPPORTED;
        }
        if (!set_lds(c->ks64.limit, c->lim_lds)) {
            delete c;
            return DG_EDEVICE;
        }
    }
    c->cfl_tiles = (int)((c->ncells + c->cfl_C - 1) / c->cfl_C);
    c->cfl_blocks = std::min(c->cfl_tiles, kCflBlocks);
    if (c->face_lds > LDS_MAX || c->cfl_lds > LDS_MAX) {
        delete c;
        return DG_EUNSUPPORTED;
    }
    const size_t lim = LDS_MAX;
    (void)set_lds(c->ks.vol, lim);
    for (int fo = 0; fo < 2; ++fo) {
        c->vol_fixed[fo] = get_vol_fixed(d, c->precision, order, c->phys, c->vol_C, c->vol_T, fo);
        if (c->vol_fixed[fo])
            (void)set_lds(c->vol_fixed[fo], lim);
    }
    (void)set_lds(c->ks.face, lim);
    c->face_fixed = get_face_fixed(d, c->precision, order, c->phys, c->face_C, c->face_T);
    if (c->face_fixed)
        (void)set_lds(c->face_fixed, lim);
    (void)set_lds(c->ks64.cfl, lim);

    // buffers
    const size_t nstate = (size_t)c->ncells * c->F * c->NM;
    const int nreg = c->stages == 1 ? 0 : c->stages == 2 ? 1 : c->stages == 3 ? 2 : 3;
    bool good = true;
    for (int i = 0; i < nreg && good; ++i) good = ok(hipMalloc(&c->reg[i], nstate * sizeof(double)));
    good = good && ok(hipMalloc(&c->fb, c->fb_bytes > 0 ? c->fb_bytes : 16));
    if (av_on)
        for (int i = 0; i < 2 && good; ++i) {
            good = ok(hipMalloc(&c->R[i], c->ncells * sizeof(double)));
            good = good && ok(hipMemset(c->R[i], 0, c->ncells * sizeof(double)));
        }
    good = good && ok(hipMalloc(&c->cfl_part, (size_t)c->cfl_tiles * 2 * sizeof(double)));
    good = good && ok(hipMalloc(&c->scal, 16 * sizeof(double)));
    good = good && ok(hipMalloc(&c->flag, sizeof(int)));
    good = good && ok(hipMemset(c->flag, 0, sizeof(int)));
    c->tot_chunk = 4096;
    c->tot_blocks = (int)((c->ncells + c->tot_chunk - 1) / c->tot_chunk);
    good = good && ok(hipMalloc(&c->tot_part, (size_t)c->tot_blocks * c->Fc * 2 * sizeof(double)));
    if (!good) {
        free_bufs(c);
        delete c;
        (void)hipGetLastError();
        return DG_ENOMEM;
    }
    if (!ok(hipDeviceSynchronize())) {
        free_bufs(c);
        delete c;
        return DG_EDEVICE;
    }
    *out = c;
    return DG_OK;
}

void dg_free(dg_ctx *ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    free_bufs(ctx);
    if (ctx->ev_pool) {
        for (hipEvent_t e : *ctx->ev_pool) (void)hipEventDestroy(e);
        delete ctx->ev_pool;
    }
    delete ctx->ev_kind;
    delete ctx;
}

dg_status dg_timing_enable(dg_ctx *c, int on)
{
    if (!c) return DG_EINVAL;
    if (on && !c->ev_pool) {
        // full capacity up front: launch() then never reallocates (nothing
        // can throw across the ABI while kernels are being recorded)
        try {
            c->ev_pool = new std::vector<hipEvent_t>();
            c->ev_kind = new std::vector<int>();
            c->ev_pool->reserve(2 * EV_MAX);
            c->ev_kind->reserve(EV_MAX);
        } catch (...) {
            delete c->ev_pool;
            delete c->ev_kind;
            c->ev_pool = nullptr;
            c->ev_kind = nullptr;
            return DG_ENOMEM;
        }
    }
    c->timing = on ? 1 : 0;
    return DG_OK;
}

dg_status dg_timing_read(dg_ctx *c, double *face_ms, long long *face_n, double *vol_ms, long long *vol_n,
                         double *cfl_ms, long long *cfl_n, long long *dropped)
{
    if (!c) return DG_EINVAL;
    double ms[3] = {0, 0, 0};
    long long n[3] = {0, 0, 0};
    if (c->ev_used > 0) {
        if (!ok(hipEventSynchronize((*c->ev_pool)[2 * c->ev_used - 1]))) return DG_EDEVICE;
        for (long long i = 0; i < c->ev_used; ++i) {
            float t = 0.0f;
            if (!ok(hipEventElapsedTime(&t, (*c->ev_pool)[2 * i], (*c->ev_pool)[2 * i + 1]))) return DG_EDEVICE;
            const int k = (*c->ev_kind)[i];
            ms[k] += t;
            ++n[k];
        }
    }
    if (face_ms) *face_ms = ms[0];
    if (face_n) *face_n = n[0];
    if (vol_ms) *vol_ms = ms[1];
    if (vol_n) *vol_n = n[1];
    if (cfl_ms) *cfl_ms = ms[2];
    if (cfl_n) *cfl_n = n[2];
    if (dropped) *dropped = c->ev_dropped;
    c->ev_used = 0;
    c->ev_dropped = 0;
    if (c->ev_kind) c->ev_kind->clear();
    return DG_OK;
}

size_t dg_state_len(const dg_ctx *c) { return c ? (size_t)c->ncells * c->F * c->NM : 0; }

int dg_num_modes(const dg_ctx *c) { return c ? c->NM : 0; }

int dg_num_fields(const dg_ctx *c) { return c ? c->F : 0; }

int dg_num_conserved(const dg_ctx *c) { return c ? c->Fc : 0; }

dg_status dg_shape(const dg_ctx *c, int *dim, int *order, long long *ncells, int *nfields)
{
    if (!c) return DG_EINVAL;
    if (dim) *dim = c->dim;
    if (order) *order = c->P;
    if (ncells) *ncells = c->ncells;
    if (nfields) *nfields = c->F;
    return DG_OK;
}

// The kernels move the state in 16-byte groups.
static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

dg_status dg_rhs(dg_ctx *c, const double *w, double *wdot, void *stream)
{
    if (!c || !w || !wdot || w == wdot || !aligned16(w) || !aligned16(wdot)) return DG_EINVAL;
    dgk::VolArgs v = blank_args();
    v.cur = w;
    v.out = wdot;
    v.c_L = 1.0;
    v.dt = 1.0;
    v.R_prev = c->ph.av_on ? c->R[c->rpar] : nullptr;
    v.check = 0;
    return stage(c, v, (hipStream_t)stream);
}

dg_status dg_step(dg_ctx *c, double *w, double dt, void *stream)
{
    if (!c || !w || !aligned16(w) || !(dt > 0.0) || !std::isfinite(dt)) return DG_EINVAL;
    return rk_step(c, w, dt, nullptr, (hipStream_t)stream);
}

dg_status dg_step_cfl(dg_ctx *c, double *w, double *dt_dev, void *stream)
{
    if (!c || !w || !aligned16(w)) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    dg_status st = run_cfl(c, w, dt_dev, s, false);
    if (st == DG_OK) st = rk_step(c, w, 0.0, c->scal, s);
    c->fin_pending = false;
    return st;
}

dg_status dg_limit(dg_ctx *c, double *w, void *stream)
{
    if (!c || !w || ((uintptr_t)w & 7)) return DG_EINVAL;
    if (!c->ks64.limit) return DG_EUNSUPPORTED;
    if (!c->limiter) {
        // limiter tiles of a context created without the option
        size_t per_cell = c->ks64.limit_lds(1, 256) - c->ks64.limit_lds(0, 256);
        c->lim_C = (int)std::max<size_t>(1, (64 * 1024) / std::max<size_t>(per_cell, 1));
        if (c->lim_C > 256) c->lim_C = 256;
        if (c->lim_C > c->ncells) c->lim_C = (int)c->ncells;
        c->lim_T = 256;
        c->lim_lds = c->ks64.limit_lds(c->lim_C, c->lim_T);
        if (c->lim_lds > LDS_MAX) return DG_EUNSUPPORTED;
        if (!set_lds(c->ks64.limit, c->lim_lds)) return DG_EDEVICE;
    }
    return run_limiter(c, w, (hipStream_t)stream);
}

dg_status dg_max_dt(dg_ctx *c, const double *w, double *dt_out, double *cmax_out, double *vmax_out, void *stream)
{
    if (!c || !w || !aligned16(w) || !dt_out) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    dg_status st = run_cfl(c, w, nullptr, s);
    if (st != DG_OK) return st;
    double res[3];
    if (!ok(hipMemcpyAsync(res, c->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s))) return DG_EDEVICE;
    if (!ok(hipStreamSynchronize(s))) return DG_EDEVICE;
    *dt_out = res[0];
    if (cmax_out) *cmax_out = res[1];
    if (vmax_out) *vmax_out = res[2];
    return DG_OK;
}

dg_status dg_max_dt_noalloc(dg_ctx *c, const double *w, double *out, void *stream)
{
    if (!c || !w || !aligned16(w) || !out || ((uintptr_t)out & 7)) return DG_EINVAL;
    int dev = -1;
    if (!ok(hipGetDevice(&dev))) return DG_EDEVICE;
    if (dev != c->device || dev < 0 || dev >= kMaxDevices || !g_scratch_dev[dev]) return DG_EINVAL;
    if (2LL * c->cfl_blocks > kScratchDoubles) return DG_ESCRATCH;
    hipStream_t s = (hipStream_t)stream;
    double *part = g_scratch_dev[dev];
    // every partial the finalize reads is written by the CFL launch before it
    // (one per block), so nothing needs clearing
    dgk::CflArgs ca;
    ca.w = w;
    ca.part = part;
    ca.cells_per_block = c->cfl_C;
    void *args[] = {&c->ph, &c->geo, &ca};
    if (!ok(hipLaunchKernel(c->ks64.cfl, dim3((unsigned)c->cfl_blocks), dim3(c->cfl_T), args, c->cfl_lds, s)))
        return DG_EDEVICE;
    double num = c->cfl * c->ph.h / (2.0 * c->P);
    const double *pp = part;
    int nblk = c->cfl_blocks;
    double *dt_copy = nullptr;
    void *fargs[] = {&pp, &nblk, &out, &dt_copy, &num};
    if (!ok(hipLaunchKernel((const void *)&cfl_finalize, dim3(1), dim3(kFinT), fargs, 0, s))) return DG_EDEVICE;
    return DG_OK;
}

dg_status dg_conserved_totals(dg_ctx *c, const double *w, double *out, void *stream)
{
    if (!c || !w || !out) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double vol = 1.0;
    for (int a = 0; a < c->dim; ++a) vol *= c->ph.h;
    {
        long long nc = c->ncells;
        int F = c->F, NP = c->NM, Fc = c->Fc, chunk = c->tot_chunk;
        double *part = c->tot_part;
        void *a1[] = {(void *)&w, &nc, &F, &NP, &Fc, &vol, &chunk, &part};
        if (!ok(hipLaunchKernel((const void *)&totals_partial, dim3(c->tot_blocks), dim3(256), a1, 0, s)))
            return DG_EDEVICE;
        int nb = c->tot_blocks;
        double *o = c->scal + 3;
        void *a2[] = {&part, &nb, &Fc, &o};
        if (!ok(hipLaunchKernel((const void *)&totals_final, dim3(1), dim3(64), a2, 0, s))) return DG_EDEVICE;
    }
    if (!ok(hipMemcpyAsync(out, c->scal + 3, c->Fc * sizeof(double), hipMemcpyDeviceToHost, s))) return DG_EDEVICE;
    if (!ok(hipStreamSynchronize(s))) return DG_EDEVICE;
    return DG_OK;
}

dg_status dg_set_forcing(dg_ctx *c, const double *s_coeffs)
{
    if (!c || ((uintptr_t)s_coeffs & 7)) return DG_EINVAL;
    if (!s_coeffs) {
        c->forcing = nullptr;
        c->forcing_src = nullptr;
        c->forcing_dirty = false;
        return DG_OK;
    }
    if (c->vol_lds_forced > LDS_MAX || !c->ks.fpts) return DG_EUNSUPPORTED;
    if (!c->spts) {
        const size_t tsz = c->precision == DG_PREC_FP64 ? sizeof(double) : sizeof(float);
        if (!ok(hipMalloc(&c->spts, (size_t)c->ncells * c->dim * c->NP * tsz))) {
            (void)hipGetLastError();
            c->spts = nullptr;
            return DG_ENOMEM;
        }
    }
    c->forcing_src = s_coeffs;
    c->forcing = c->spts;
    c->forcing_dirty = true;
    return DG_OK;
}

dg_status dg_set_sensor_rate(dg_ctx *c, const double *R, void *stream)
{
    if (!c || !R || !c->ph.av_on) return DG_EINVAL;
    if (!ok(hipMemcpyAsync(c->R[c->rpar], R, c->ncells * sizeof(double), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream)))
        return DG_EDEVICE;
    return DG_OK;
}

dg_status dg_get_sensor_rate(dg_ctx *c, double *R, void *stream)
{
    if (!c || !R || !c->ph.av_on) return DG_EINVAL;
    if (!ok(hipMemcpyAsync(R, c->R[c->rpar], c->ncells * sizeof(double), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream)))
        return DG_EDEVICE;
    return DG_OK;
}

dg_status dg_check(dg_ctx *c, void *stream)
{
    if (!c) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int f = 0;
    if (!ok(hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, s))) return DG_EDEVICE;
    if (!ok(hipStreamSynchronize(s))) return DG_EDEVICE;
    if (f) {
        if (!ok(hipMemsetAsync(c->flag, 0, sizeof(int), s))) return DG_EDEVICE;
        if (!ok(hipStreamSynchronize(s))) return DG_EDEVICE;
    }
    if (f & 2) return DG_ENONFINITE;
    if (f & 1) return DG_ENONPHYSICAL;
    return DG_OK;
}

dg_status dg_get_tiles(const dg_ctx *c, int *vol_cells, int *vol_threads, int *face_cells, int *face_threads)
{
    if (!c) return DG_EINVAL;
    if (vol_cells) *vol_cells = c->vol_C;
    if (vol_threads) *vol_threads = c->vol_T;
    if (face_cells) *face_cells = c->face_C;
    if (face_threads) *face_threads = c->face_T;
    return DG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched ensembles
// ---------------------------------------------------------------------------

namespace {

struct Group {
    int P = 0;
    std::vector<int> boxes;                 // box ids of this order
    std::vector<dgk::BoxDesc> h_desc;
    dgk::BoxDesc *d_desc = nullptr;
    KernelSet ks{}, ks64{};
    long long nblk[3] = {0, 0, 0};          // total flat blocks per kind
    int vol_T = 0, face_T = 0, cfl_T = 0;
    size_t vol_lds = 0, face_lds = 0, cfl_lds = 0;
    int stages = 0;
};

}  // namespace

struct dg_batch {
    int nbox = 0, dim = 0;
    double cfl = 0.5;
    std::vector<dg_ctx *> box;
    std::vector<Group> groups;
    std::vector<int> large;        // boxes stepped by their own kernels inside the step
    std::vector<double *> wptr;
    const double *dt_in = nullptr; // caller's per-box step sizes (device) of the step being enqueued, or null (CFL)
    const double *graph_dt = nullptr;   // dt_in of the captured graph
    bool have_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;     // private stream for graph capture
    // independent units (each large box, each order group) run on their own
    // streams, forked from and joined back to the step's stream: parallel
    // branches of the captured graph
    std::vector<hipStream_t> ustream;
    std::vector<hipEvent_t> uevent;
    hipEvent_t fork = nullptr;
};

namespace {

void batch_release(dg_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipStream_t st : b->ustream)
        if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t e : b->uevent)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (Group &g : b->groups)
        if (g.d_desc) (void)hipFree(g.d_desc);
    for (dg_ctx *c : b->box) dg_free(c);
}

// Shu-Osher stage table for a scheme with S stages, register roles
// (0 = state, 1..3 = RK registers), identical to rk_step.
int stage_table(int S, dgk::StageDesc *sd)
{
    auto mk = [](int cur, int base, int out, double cb, double cc, double cl) {
        dgk::StageDesc d;
        d.cur = cur;
        d.base = base;
        d.x2 = -1;
        d.out = out;
        d.out2 = -1;
        d.c_base = cb;
        d.c_cur = cc;
        d.c_L = cl;
        d.d_x2 = d.d_cur = d.d_L = 0.0;
        return d;
    };
    if (S == 1) {
        sd[0] = mk(0, -1, 0, 0.0, 1.0, 1.0);
        return 1;
    }
    if (S == 2) {
        sd[0] = mk(0, -1, 1, 0.0, 1.0, 1.0);
        sd[1] = mk(1, 0, 0, 0.5, 0.5, 0.5);
        return 2;
    }
    if (S == 3) {
        sd[0] = mk(0, -1, 1, 0.0, 1.0, 1.0);
        sd[1] = mk(1, 0, 2, 0.75, 0.25, 0.25);
        sd[2] = mk(2, 0, 0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0);
        return 3;
    }
    sd[0] = mk(0, -1, 1, 0.0, 1.0, 0.391752226571890);
    sd[1] = mk(1, 0, 2, 0.444370493651235, 0.555629506348765, 0.368410593050371);
    sd[2] = mk(2, 0, 3, 0.620101851488403, 0.379898148511597, 0.251891774271694);
    sd[3] = mk(3, 0, 1, 0.178079954393132, 0.821920045606868, 0.544974750228521);
    sd[3].out2 = 0;
    sd[3].x2 = 2;
    sd[3].d_x2 = 0.517231671970585;
    sd[3].d_cur = 0.096059710526147;
    sd[3].d_L = 0.063692468666290;
    sd[4] = mk(1, 0, 0, 1.0, 0.386708617503269, 0.226007483236906);
    return 5;
}

// Boxes with at least this many cells keep their own (fixed-tile) kernels
// inside the batched step: they fill the device by themselves, and the grouped
// kernels' per-block box lookup only pays off for the small, launch-bound ones.
constexpr long long kBatchLargeCells = 65536;

// Streams over which the independent units of a batched step are spread.
constexpr int kBatchStreams = 8;

// The step of one unit: a large box (its own kernels) or an order group
// (grouped launches over its boxes), all on stream s.
dg_status unit_enqueue(dg_batch *b, int u, hipStream_t s)
{
    if (u < (int)b->large.size()) {
        const int i = b->large[u];
        dg_ctx *c = b->box[i];
        dg_status st = DG_OK;
        if (b->dt_in) {
            const double *src = b->dt_in + i;
            double *dst = c->scal;
            void *args[] = {&src, &dst};
            if (!ok(hipLaunchKernel((const void *)&dt_in_single, dim3(1), dim3(64), args, 0, s))) return DG_EDEVICE;
        } else {
            st = run_cfl(c, b->wptr[i], nullptr, s, false);
        }
        if (st == DG_OK) st = rk_step(c, b->wptr[i], 0.0, c->scal, s);
        c->fin_pending = false;
        return st;
    }
    {
        Group &g = b->groups[u - b->large.size()];
        const int n = (int)g.boxes.size();
        dgk::BoxDesc *d = g.d_desc;
        if (b->dt_in) {
            const double *src = b->dt_in;
            void *args[] = {&d, (void *)&n, &src};
            if (!ok(hipLaunchKernel((const void *)&dt_in_batched, dim3((unsigned)((n + 63) / 64)), dim3(64), args, 0,
                                    s)))
                return DG_EDEVICE;
        } else {
            {
                void *args[] = {&d, (void *)&n};
                if (!ok(hipLaunchKernel(g.ks64.cfl_b, dim3((unsigned)g.nblk[2]), dim3(g.cfl_T), args, g.cfl_lds, s)))
                    return DG_EDEVICE;
            }
            double cfl = b->cfl;
            void *args[] = {&d, &cfl};
            if (!ok(hipLaunchKernel((const void *)&cfl_finalize_batched, dim3(n), dim3(kFinT), args, 0, s)))
                return DG_EDEVICE;
        }
        dgk::StageDesc sd[5];
        const int S = stage_table(g.stages, sd);
        for (int k = 0; k < S; ++k) {
            int cur = sd[k].cur;
            void *fargs[] = {&d, (void *)&n, &cur};
            if (!ok(hipLaunchKernel(g.ks.face_b, dim3((unsigned)g.nblk[1]), dim3(g.face_T), fargs, g.face_lds, s)))
                return DG_EDEVICE;
            void *vargs[] = {&d, (void *)&n, &sd[k]};
            if (!ok(hipLaunchKernel(g.ks.vol_b, dim3((unsigned)g.nblk[0]), dim3(g.vol_T), vargs, g.vol_lds, s)))
                return DG_EDEVICE;
        }
    }
    return DG_OK;
}

// The whole batched step on stream s: every unit on its own stream (round
// robin over the batch's streams), forked from s by an event and joined back
// by one event per unit, so that independent boxes overlap on the device.
dg_status batch_enqueue(dg_batch *b, hipStream_t s)
{
    const int nu = (int)(b->large.size() + b->groups.size());
    const int ns = (int)b->ustream.size();
    if (ns == 0) {
        for (int u = 0; u < nu; ++u) {
            dg_status st = unit_enqueue(b, u, s);
            if (st != DG_OK) return st;
        }
        return DG_OK;
    }
    if (!ok(hipEventRecord(b->fork, s))) return DG_EDEVICE;
    for (int k = 0; k < ns; ++k)
        if (!ok(hipStreamWaitEvent(b->ustream[k], b->fork, 0))) return DG_EDEVICE;
    for (int u = 0; u < nu; ++u) {
        dg_status st = unit_enqueue(b, u, b->ustream[u % ns]);
        if (st != DG_OK) return st;
    }
    for (int k = 0; k < ns; ++k) {
        if (!ok(hipEventRecord(b->uevent[k], b->ustream[k]))) return DG_EDEVICE;
        if (!ok(hipStreamWaitEvent(s, b->uevent[k], 0))) return DG_EDEVICE;
    }
    return DG_OK;
}

}  // namespace

extern "C" {

static dg_status batch_init_impl(int nbox, const dg_mesh *meshes, const int *orders, double gamma, double nu, double kappa,
                               const dg_av_params *av, const dg_options *opt, dg_batch **out)
{
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (nbox < 1 || !meshes || !orders) return DG_EINVAL;
    if (av && av->enabled) return DG_EUNSUPPORTED;
    if (opt && (opt->limiter || opt->tracer || opt->basis)) return DG_EUNSUPPORTED;
    for (int i = 0; i < nbox; ++i)
        if (meshes[i].dim != meshes[0].dim) return DG_EINVAL;
    dg_batch *b = new (std::nothrow) dg_batch;
    if (!b) return DG_ENOMEM;
    // releases the partly built batch (every box context initialised so far
    // and every group table allocated so far) on each early return and on an
    // exception; disarmed once the batch is complete
    struct Guard {
        dg_batch *b;
        ~Guard()
        {
            if (b) {
                batch_release(b);
                delete b;
            }
        }
    } guard{b};
    b->nbox = nbox;
    b->dim = meshes[0].dim;
    b->cfl = opt ? opt->cfl : 0.5;
    b->box.assign(nbox, nullptr);
    b->wptr.assign(nbox, nullptr);
    for (int i = 0; i < nbox; ++i) {
        dg_status st = dg_init(&meshes[i], orders[i], gamma, nu, kappa, nullptr, opt, &b->box[i]);
        if (st != DG_OK) {
            return st;
        }
    }
    for (int i = 0; i < nbox; ++i)
        if (b->box[i]->ncells >= kBatchLargeCells) b->large.push_back(i);
    for (int P = 1; P <= MAXP; ++P) {
        Group g;
        g.P = P;
        for (int i = 0; i < nbox; ++i)
            if (orders[i] == P && b->box[i]->ncells < kBatchLargeCells) g.boxes.push_back(i);
        if (g.boxes.empty()) continue;
        const dg_ctx *c0 = b->box[g.boxes[0]];
        g.ks = c0->ks;
        g.ks64 = c0->ks64;
        g.vol_T = c0->vol_T;
        g.face_T = c0->face_T;
        g.cfl_T = c0->cfl_T;
        g.vol_lds = c0->vol_lds;
        g.face_lds = c0->face_lds;
        g.cfl_lds = c0->cfl_lds;
        g.stages = c0->stages;
        // fixed-tile grouped kernels when the (common) tile has one
        {
            const void *vf = get_vol_fixed(c0->dim, c0->precision, P, c0->phys, c0->vol_C, c0->vol_T, 0, 1);
            const void *ff = get_face_fixed(c0->dim, c0->precision, P, c0->phys, c0->face_C, c0->face_T, 1);
            if (vf) g.ks.vol_b = vf;
            if (ff) g.ks.face_b = ff;
        }
        if (!g.ks.vol_b || !g.ks.face_b || !g.ks64.cfl_b) {
            return DG_EUNSUPPORTED;
        }
        (void)set_lds(g.ks.vol_b, LDS_MAX);
        (void)set_lds(g.ks.face_b, LDS_MAX);
        (void)set_lds(g.ks64.cfl_b, LDS_MAX);
        for (int i : g.boxes) {
            const dg_ctx *c = b->box[i];
            dgk::BoxDesc d;
            memset(&d, 0, sizeof(d));
            d.ph = c->ph;
            d.geo = c->geo;
            d.reg[0] = nullptr;
            for (int r = 0; r < 3; ++r) d.reg[1 + r] = c->reg[r];
            d.fb = c->fb;
            d.cfl_part = c->cfl_part;
            d.dt = c->scal;
            d.flag = c->flag;
            d.cells_per_block = c->vol_C;
            d.faces_per_block = c->face_C;
            d.cfl_cells = c->cfl_C;
            d.bidx = i;
            d.nblocks[0] = (c->ncells + c->vol_C - 1) / c->vol_C;
            long long nf = 0;
            for (int a = 0; a < c->dim; ++a) {
                long long np = (c->geo.nf[a] + c->face_C - 1) / c->face_C;
                for (int q = 0; q < 3; ++q)
                    if (q != a) np *= c->geo.n[q];
                nf += np;
            }
            d.nblocks[1] = nf;
            d.nblocks[2] = c->cfl_tiles;
            for (int k = 0; k < 3; ++k) {
                d.start[k] = g.nblk[k];
                g.nblk[k] += d.nblocks[k];
            }
            g.h_desc.push_back(d);
        }
        // owned by the batch before the allocation, so that the guard frees it
        b->groups.push_back(g);
        Group &gb = b->groups.back();
        if (!ok(hipMalloc(&gb.d_desc, sizeof(dgk::BoxDesc) * gb.h_desc.size()))) {
            gb.d_desc = nullptr;
            (void)hipGetLastError();
            return DG_ENOMEM;
        }
    }
    // streams for the independent units (default priority, non-blocking)
    {
        const int nu = (int)(b->large.size() + b->groups.size());
        const int ns = std::min(nu, kBatchStreams);
        if (ns > 1) {
            if (!ok(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming))) return DG_EDEVICE;
            for (int k = 0; k < ns; ++k) {
                hipStream_t st = nullptr;
                hipEvent_t ev = nullptr;
                if (!ok(hipStreamCreateWithFlags(&st, hipStreamNonBlocking))) return DG_EDEVICE;
                b->ustream.push_back(st);
                if (!ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming))) return DG_EDEVICE;
                b->uevent.push_back(ev);
            }
        }
    }
    guard.b = nullptr;
    *out = b;
    return DG_OK;
}

dg_status dg_batch_init(int nbox, const dg_mesh *meshes, const int *orders, double gamma, double nu, double kappa,
                        const dg_av_params *av, const dg_options *opt, dg_batch **out)
{
    try {
        return batch_init_impl(nbox, meshes, orders, gamma, nu, kappa, av, opt, out);
    } catch (...) {   // host allocations; nothing throws across the ABI
        if (out) *out = nullptr;
        return DG_ENOMEM;
    }
}

void dg_batch_free(dg_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_release(b);
    delete b;
}

namespace {

// dg_batch_step (dt_dev = null: per-box CFL steps) and dg_batch_step_dt.
dg_status batch_step(dg_batch *b, double *const *w, const double *dt_dev, int use_graph, void *stream)
{
    if (!b || !w || ((uintptr_t)dt_dev & 7)) return DG_EINVAL;
    for (int i = 0; i < b->nbox; ++i)
        if (!w[i] || !aligned16(w[i])) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    b->dt_in = dt_dev;
    bool changed = b->have_graph && b->graph_dt != dt_dev;   // another step-size source: capture again
    for (int i = 0; i < b->nbox; ++i)
        if (b->wptr[i] != w[i]) changed = true;
    if (changed) {
        for (int i = 0; i < b->nbox; ++i) b->wptr[i] = w[i];
        for (Group &g : b->groups) {
            for (size_t k = 0; k < g.boxes.size(); ++k) g.h_desc[k].reg[0] = w[g.boxes[k]];
            if (!ok(hipMemcpyAsync(g.d_desc, g.h_desc.data(), sizeof(dgk::BoxDesc) * g.h_desc.size(),
                                   hipMemcpyHostToDevice, s)))
                return DG_EDEVICE;
        }
        if (!ok(hipStreamSynchronize(s))) return DG_EDEVICE;
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->have_graph = false;
    }
    if (!use_graph) return batch_enqueue(b, s);
    if (!b->have_graph) {
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph is launched on the caller's
        if (!b->cap && !ok(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking))) return DG_EDEVICE;
        if (!ok(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed))) return DG_EDEVICE;
        dg_status st = batch_enqueue(b, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (st != DG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (!ok(e) || !g) return DG_EDEVICE;
        hipGraphExec_t ex = nullptr;
        if (!ok(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0))) {
            (void)hipGraphDestroy(g);
            return DG_EDEVICE;
        }
        b->graph = g;
        b->exec = ex;
        b->have_graph = true;
        b->graph_dt = dt_dev;
    }
    return ok(hipGraphLaunch(b->exec, s)) ? DG_OK : DG_EDEVICE;
}

}  // namespace

dg_status dg_batch_step(dg_batch *b, double *const *w, int use_graph, void *stream)
{
    return batch_step(b, w, nullptr, use_graph, stream);
}

dg_status dg_batch_step_dt(dg_batch *b, double *const *w, const double *dt_dev, int use_graph, void *stream)
{
    if (!dt_dev) return DG_EINVAL;
    return batch_step(b, w, dt_dev, use_graph, stream);
}

dg_status dg_batch_dt(dg_batch *b, double *dt_out, void *stream)
{
    if (!b || !dt_out) return DG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < b->nbox; ++i)
        if (!ok(hipMemcpyAsync(&dt_out[i], b->box[i]->scal, sizeof(double), hipMemcpyDeviceToHost, s)))
            return DG_EDEVICE;
    return ok(hipStreamSynchronize(s)) ? DG_OK : DG_EDEVICE;
}

int dg_batch_size(const dg_batch *b) { return b ? b->nbox : 0; }

dg_status dg_batch_box(dg_batch *b, int i, dg_ctx **ctx)
{
    if (!b || !ctx || i < 0 || i >= b->nbox) return DG_EINVAL;
    *ctx = b->box[i];
    return DG_OK;
}

}  // extern "C"
