// dg_forcing.hip -- the driving field of the turbulence problem (Sec. 7.1):
// Fourier modes on the band 1 <= |k| <= k_max whose complex amplitudes follow
// an Ornstein-Uhlenbeck process with a k^(-5/3) spectrum and are kept
// solenoidal (host, FP64), and the projection of the field
// s(x) = sum_k 2 Re(a_k exp(2 pi i k.x)) on the per-cell Legendre basis
// (device kernel, FP64).  The RHS reads the projected coefficients through
// dg_set_forcing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "dg.h"

namespace {

typedef long double LD;

// Scaled Legendre values Pt_l(x) = sqrt(2l+1) P_l(x), l <= lmax (Bonnet).
void sleg(int lmax, LD x, LD *P)
{
    LD a = 1.0L, b = x;
    P[0] = 1.0L;
    if (lmax >= 1) P[1] = x;
    for (int l = 1; l < lmax; ++l) {
        const LD c = ((2 * l + 1) * x * b - l * a) / (l + 1);
        a = b;
        b = c;
        P[l + 1] = c;
    }
    for (int l = 0; l <= lmax; ++l) P[l] *= sqrtl(2.0L * l + 1.0L);
}

// n-point Gauss-Legendre rule (Newton on P_n).
void gauss(int n, LD *x, LD *w)
{
    for (int i = 0; i < n; ++i) {
        LD z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 60; ++it) {
            LD p0 = 1.0L, p1 = z;
            for (int l = 1; l < n; ++l) {
                const LD p2 = ((2 * l + 1) * z * p1 - l * p0) / (l + 1);
                p0 = p1;
                p1 = p2;
            }
            const LD dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const LD dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        LD p0 = 1.0L, p1 = z;
        for (int l = 1; l < n; ++l) {
            const LD p2 = ((2 * l + 1) * z * p1 - l * p0) / (l + 1);
            p0 = p1;
            p1 = p2;
        }
        const LD dp = n * (z * p1 - p0) / (z * z - 1.0L);
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

constexpr int kMaxK = 4;      // largest supported k_max
constexpr int kMaxP = 8;

}  // namespace

struct dg_forcing {
    int dim, P, NP;    // NP: stored modes per component (p^dim, or the total-degree count)
    int basis;
    int n[3];
    double lo[3], h;
    long long ncells;
    int kmax, nm;
    double t_corr, sigma0;
    std::vector<int> kv;          // [nm][3]
    std::vector<double> amp;      // [nm][3][2]
    std::vector<double> tab;      // device table image: k, amplitudes, J
    double *d_tab;
    size_t tab_len;
};

namespace {

// Host image of the device table: k as doubles [nm][3], amplitudes [nm][3][2],
// J[k_a + kmax][l][2] = (1/2) int_{-1}^{1} exp(i pi k_a h xi) Pt_l(xi) dxi,
// the 1D factor of a mode's projection on a cell (the cell-centre phase apart).
void build_static(dg_forcing *f)
{
    const int nk = 2 * f->kmax + 1;
    f->tab_len = (size_t)f->nm * 3 + (size_t)f->nm * 6 + (size_t)nk * f->P * 2;
    f->tab.assign(f->tab_len, 0.0);
    for (int i = 0; i < f->nm; ++i)
        for (int a = 0; a < 3; ++a) f->tab[i * 3 + a] = (double)f->kv[i * 3 + a];
    double *J = f->tab.data() + (size_t)f->nm * 9;
    LD xq[48], wq[48], Pt[kMaxP + 1];
    gauss(48, xq, wq);
    for (int ka = -f->kmax; ka <= f->kmax; ++ka)
        for (int l = 0; l < f->P; ++l) {
            LD re = 0.0L, im = 0.0L;
            for (int q = 0; q < 48; ++q) {
                sleg(f->P - 1, xq[q], Pt);
                const LD th = 3.14159265358979323846264338327950288L * ka * (LD)f->h * xq[q];
                re += 0.5L * wq[q] * cosl(th) * Pt[l];
                im += 0.5L * wq[q] * sinl(th) * Pt[l];
            }
            J[((ka + f->kmax) * f->P + l) * 2] = (double)re;
            J[((ka + f->kmax) * f->P + l) * 2 + 1] = (double)im;
        }
}

// s[(cell * D + c) * NP + m] = sum_i 2 Re(a_ic prod_a e^{2 pi i k_ia x_ca} J(k_ia, l_a)),
// one thread per (cell, stored mode m): m = l_x + p (l_y + p l_z) for the
// tensor basis; for the total-degree basis the modes of degree <= p - 1 in
// the order l_z, l_y, l_x ascending (l_x fastest).
template <int D>
__device__ __forceinline__ void project_item(const double *__restrict__ tab, int nm, int kmax, int P, int NP,
                                             int basis, int n0, int n1, double lo0, double lo1, double lo2, double h,
                                             long long item, double *__restrict__ s);

// Grid-stride over the (cell, mode) items, so that any mesh fits a grid of
// at most 2^20 blocks.  The table (tab_len doubles) is staged in LDS first:
// every item reads all of it.
template <int D>
__global__ void __launch_bounds__(256) forcing_project_kernel(const double *__restrict__ tab, int tab_len, int nm,
                                                              int kmax, int P, int NP, int basis, int n0, int n1,
                                                              double lo0, double lo1, double lo2, double h,
                                                              long long ncells, double *__restrict__ s)
{
    extern __shared__ double tl[];
    for (int i = threadIdx.x; i < tab_len; i += blockDim.x) tl[i] = tab[i];
    __syncthreads();
    const long long total = ncells * NP;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x; item < total; item += stride)
        project_item<D>(tl, nm, kmax, P, NP, basis, n0, n1, lo0, lo1, lo2, h, item, s);
}

template <int D>
__device__ __forceinline__ void project_item(const double *__restrict__ tab, int nm, int kmax, int P, int NP,
                                             int basis, int n0, int n1, double lo0, double lo1, double lo2, double h,
                                             long long item, double *__restrict__ s)
{
    const long long cell = item / NP;
    const int m = (int)(item - cell * NP);
    int l[3] = {m % P, (m / P) % P, m / (P * P)};
    if (basis == 1) {
        int r = m;
        l[0] = l[1] = l[2] = 0;
        for (int lz = 0; lz < (D == 3 ? P : 1); ++lz)
            for (int ly = 0; ly < P - lz; ++ly) {
                const int nl = P - ly - lz;
                if (r >= 0 && r < nl) {
                    l[0] = r;
                    l[1] = ly;
                    l[2] = lz;
                }
                r -= nl;
            }
    }
    const long long r0 = cell / n0;
    const int ijk[3] = {(int)(cell - r0 * n0), (int)(r0 % n1), (int)(r0 / n1)};
    const double lo[3] = {lo0, lo1, lo2};
    // powers e^{2 pi i k x_c}, k = 0..kmax, per axis
    double pr[3][kMaxK + 1], pim[3][kMaxK + 1];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double xc = lo[a] + (ijk[a] + 0.5) * h;
        double sn, cs;
        sincospi(2.0 * xc, &sn, &cs);
        pr[a][0] = 1.0;
        pim[a][0] = 0.0;
        for (int k = 1; k <= kmax; ++k) {
            pr[a][k] = pr[a][k - 1] * cs - pim[a][k - 1] * sn;
            pim[a][k] = pr[a][k - 1] * sn + pim[a][k - 1] * cs;
        }
    }
    const double *kvd = tab;
    const double *am = tab + (size_t)nm * 3;
    const double *J = tab + (size_t)nm * 9;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < nm; ++i) {
        double er = 1.0, ei = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int ka = (int)kvd[i * 3 + a];
            const int kk = ka < 0 ? -ka : ka;
            const double zr = pr[a][kk], zi = ka < 0 ? -pim[a][kk] : pim[a][kk];
            const double jr = J[((ka + kmax) * P + l[a]) * 2], ji = J[((ka + kmax) * P + l[a]) * 2 + 1];
            const double fr = zr * jr - zi * ji, fi = zr * ji + zi * jr;
            const double tr = er * fr - ei * fi;
            ei = er * fi + ei * fr;
            er = tr;
        }
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += 2.0 * (am[(i * 3 + c) * 2] * er - am[(i * 3 + c) * 2 + 1] * ei);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) s[(cell * D + c) * NP + m] = acc[c];
}

}  // namespace

extern "C" {

dg_status dg_forcing_init(const dg_mesh *mesh, int order, int basis, int kmax, double t_corr, double sigma0,
                          dg_forcing **out)
{
    if (!out) return DG_EINVAL;
    *out = nullptr;
    if (!mesh || (mesh->dim != 2 && mesh->dim != 3) || order < 1 || order > kMaxP) return DG_EINVAL;
    if (basis != 0 && basis != 1) return DG_EINVAL;
    if (kmax < 1 || kmax > kMaxK || !(t_corr > 0.0) || !(sigma0 >= 0.0) || !std::isfinite(sigma0)) return DG_EINVAL;
    const int d = mesh->dim;
    double h = 0.0;
    long long cells = 1;
    for (int a = 0; a < d; ++a) {
        if (mesh->n[a] < 1 || !(mesh->hi[a] > mesh->lo[a])) return DG_EINVAL;
        const double ha = (mesh->hi[a] - mesh->lo[a]) / mesh->n[a];
        if (a == 0)
            h = ha;
        else if (fabs(ha - h) > 1e-12 * h)
            return DG_EINVAL;
        cells *= mesh->n[a];
    }
    dg_forcing *f = new (std::nothrow) dg_forcing;
    if (!f) return DG_ENOMEM;
    try {
        f->dim = d;
        f->P = order;
        f->basis = basis;
        f->NP = 1;
        for (int a = 0; a < d; ++a) f->NP *= order;
        if (basis == 1) f->NP = d == 2 ? order * (order + 1) / 2 : order * (order + 1) * (order + 2) / 6;
        for (int a = 0; a < 3; ++a) {
            f->n[a] = a < d ? mesh->n[a] : 1;
            f->lo[a] = a < d ? mesh->lo[a] : 0.0;
        }
        f->h = h;
        f->ncells = cells;
        f->kmax = kmax;
        f->t_corr = t_corr;
        f->sigma0 = sigma0;
        f->d_tab = nullptr;
        // modes: integer k with 1 <= |k|^2 <= kmax^2, the one of each +-k pair
        // whose first non-zero component is positive, k_x then k_y then k_z
        // ascending (k_z = 0 in 2D)
        const int kzm = d == 3 ? kmax : 0;
        for (int kx = -kmax; kx <= kmax; ++kx)
            for (int ky = -kmax; ky <= kmax; ++ky)
                for (int kz = -kzm; kz <= kzm; ++kz) {
                    const int k2 = kx * kx + ky * ky + kz * kz;
                    const int lead = kx != 0 ? kx : (ky != 0 ? ky : kz);
                    if (k2 < 1 || k2 > kmax * kmax || lead < 0) continue;
                    f->kv.push_back(kx);
                    f->kv.push_back(ky);
                    f->kv.push_back(kz);
                }
        f->nm = (int)(f->kv.size() / 3);
        f->amp.assign((size_t)f->nm * 6, 0.0);
        build_static(f);
    } catch (...) {
        delete f;
        return DG_ENOMEM;
    }
    *out = f;
    return DG_OK;
}

void dg_forcing_free(dg_forcing *f)
{
    if (!f) return;
    if (f->d_tab) {
        (void)hipDeviceSynchronize();
        (void)hipFree(f->d_tab);
    }
    delete f;
}

int dg_forcing_num_modes(const dg_forcing *f) { return f ? f->nm : 0; }

dg_status dg_forcing_modes(const dg_forcing *f, int *kv)
{
    if (!f || !kv) return DG_EINVAL;
    memcpy(kv, f->kv.data(), sizeof(int) * f->kv.size());
    return DG_OK;
}

dg_status dg_forcing_get_amplitudes(const dg_forcing *f, double *amp)
{
    if (!f || !amp) return DG_EINVAL;
    memcpy(amp, f->amp.data(), sizeof(double) * f->amp.size());
    return DG_OK;
}

dg_status dg_forcing_set_amplitudes(dg_forcing *f, const double *amp)
{
    if (!f || !amp) return DG_EINVAL;
    for (size_t i = 0; i < f->amp.size(); ++i)
        if (!std::isfinite(amp[i])) return DG_EINVAL;
    memcpy(f->amp.data(), amp, sizeof(double) * f->amp.size());
    return DG_OK;
}

dg_status dg_forcing_update(dg_forcing *f, const double *noise, double dt)
{
    if (!f || !noise || !(dt > 0.0)) return DG_EINVAL;
    for (int i = 0; i < f->nm * 6; ++i)
        if (!std::isfinite(noise[i])) return DG_EINVAL;
    const double decay = std::exp(-dt / f->t_corr);   // 0 for dt = +inf: a stationary draw
    const double kick = std::sqrt(1.0 - decay * decay) / std::sqrt(2.0);
    for (int i = 0; i < f->nm; ++i) {
        const double k[3] = {(double)f->kv[i * 3], (double)f->kv[i * 3 + 1], (double)f->kv[i * 3 + 2]};
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double sig = f->sigma0 * std::pow(k2, -5.0 / 6.0);   // sigma0 |k|^(-5/3)
        double *a = f->amp.data() + (size_t)i * 6;
        const double *xi = noise + (size_t)i * 6;
        for (int c = 0; c < f->dim; ++c)
            for (int r = 0; r < 2; ++r) a[c * 2 + r] = decay * a[c * 2 + r] + sig * kick * xi[c * 2 + r];
        // solenoidal: remove the component along k (real and imaginary parts)
        for (int r = 0; r < 2; ++r) {
            double kd = 0.0;
            for (int c = 0; c < f->dim; ++c) kd += k[c] * a[c * 2 + r];
            for (int c = 0; c < f->dim; ++c) a[c * 2 + r] -= k[c] * kd / k2;
        }
    }
    return DG_OK;
}

dg_status dg_forcing_project(dg_forcing *f, double *s, void *stream)
{
    if (!f || !s || ((uintptr_t)s & 7)) return DG_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (!f->d_tab) {
        if (hipMalloc(&f->d_tab, sizeof(double) * f->tab_len) != hipSuccess) {
            (void)hipGetLastError();
            f->d_tab = nullptr;
            return DG_ENOMEM;
        }
    }
    // current amplitudes into the table image, then to the device; the copy
    // completes before the call returns (pageable source), so the host image
    // may change afterwards
    memcpy(f->tab.data() + (size_t)f->nm * 3, f->amp.data(), sizeof(double) * f->amp.size());
    if (hipMemcpyAsync(f->d_tab, f->tab.data(), sizeof(double) * f->tab_len, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return DG_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return DG_EDEVICE;
    const long long items = f->ncells * f->NP;
    const long long blocks = (items + 255) / 256;
    const dim3 grid((unsigned)(blocks < (1LL << 20) ? blocks : (1LL << 20))), block(256);
    const void *fn = f->dim == 2 ? (const void *)&forcing_project_kernel<2> : (const void *)&forcing_project_kernel<3>;
    const double *t = f->d_tab;
    int tl = (int)f->tab_len;
    int nm = f->nm, kmax = f->kmax, P = f->P, NP = f->NP, basis = f->basis, n0 = f->n[0], n1 = f->n[1];
    double lo0 = f->lo[0], lo1 = f->lo[1], lo2 = f->lo[2], h = f->h;
    long long nc = f->ncells;
    void *args[] = {&t, &tl, &nm, &kmax, &P, &NP, &basis, &n0, &n1, &lo0, &lo1, &lo2, &h, &nc, &s};
    if (hipLaunchKernel(fn, grid, block, args, sizeof(double) * f->tab_len, st) != hipSuccess) return DG_EDEVICE;
    return DG_OK;
}

}  // extern "C"
