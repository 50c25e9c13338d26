// Kernel instantiations: dim = 2, bulk precision double, orders 1..8.
#include "dg_kernels.hpp"
#include "dg_registry.hpp"

namespace dgk {

namespace {
template <int P, bool G>
void fill(KernelSet *k)
{
    k->vol = (const void *)&vol_kernel<2, P, double, G>;
    k->face = (const void *)&face_kernel<2, P, double, G>;
    k->vol_lds = &vol_lds_bytes<2, P, double>;
    k->face_lds = &face_lds_bytes<2, P, double, G>;
    k->cfl = (const void *)&cfl_kernel<2, P>;
    k->cfl_lds = &cfl_lds_bytes<2, P>;
}

template <int P>
void pick(bool grad, KernelSet *k)
{
    if (grad)
        fill<P, true>(k);
    else
        fill<P, false>(k);
}
}  // namespace

void dgk_get_2d_f64(int P, bool grad, KernelSet *k)
{
    switch (P) {
    case 1: pick<1>(grad, k); break;
    case 2: pick<2>(grad, k); break;
    case 3: pick<3>(grad, k); break;
    case 4: pick<4>(grad, k); break;
    case 5: pick<5>(grad, k); break;
    case 6: pick<6>(grad, k); break;
    case 7: pick<7>(grad, k); break;
    case 8: pick<8>(grad, k); break;
    default: *k = KernelSet{};
    }
}

int dgk_upload_2d_f64(const Tab<double> *d, const Tab<float> *f)
{
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabd), d, sizeof(Tab<double>) * (MAXP + 1)) != hipSuccess) return -1;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabf), f, sizeof(Tab<float>) * (MAXP + 1)) != hipSuccess) return -1;
    return 0;
}

}  // namespace dgk
