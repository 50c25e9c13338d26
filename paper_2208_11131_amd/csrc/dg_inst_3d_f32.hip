// Kernel instantiations: dim = 3, bulk precision float, orders 1..8,
// physics variants Euler / Navier-Stokes / artificial viscosity /
// Navier-Stokes with the passive tracer, and the same four on the
// total-degree basis.
#include "dg_kernels.hpp"
#include "dg_registry.hpp"

namespace dgk {

namespace {
template <int P, int PH>
void fill(KernelSet *k)
{
    k->vol = (const void *)&vol_kernel<3, P, float, PH>;
    k->face = (const void *)&face_kernel<3, P, float, PH>;
    k->vol_b = (const void *)&vol_kernel_batched<3, P, float, PH>;
    k->face_b = (const void *)&face_kernel_batched<3, P, float, PH>;
    k->vol_lds = &vol_lds_bytes<3, P, float, PH>;
    k->face_lds = &face_lds_bytes<3, P, float, PH>;
    k->cfl = nullptr;
    k->cfl_b = nullptr;
    k->cfl_lds = nullptr;
    k->limit = nullptr;
    k->limit_lds = nullptr;
    k->fpts = (const void *)&forcing_points_kernel<3, P, float, Fld<3, PH>::PN>;
}

template <int P>
void pick(int ph, KernelSet *k)
{
    if (ph == 0)
        fill<P, 0>(k);
    else if (ph == 1)
        fill<P, 1>(k);
    else if (ph == 2)
        fill<P, 2>(k);
    else if (ph == 3)
        fill<P, 3>(k);
    else if (ph == 4)
        fill<P, 4>(k);
    else if (ph == 5)
        fill<P, 5>(k);
    else if (ph == 6)
        fill<P, 6>(k);
    else
        fill<P, 7>(k);
}
}  // namespace

void dgk_get_3d_f32(int P, int ph, KernelSet *k)
{
    switch (P) {
    case 1: pick<1>(ph, k); break;
    case 2: pick<2>(ph, k); break;
    case 3: pick<3>(ph, k); break;
    case 4: pick<4>(ph, k); break;
    case 5: pick<5>(ph, k); break;
    case 6: pick<6>(ph, k); break;
    case 7: pick<7>(ph, k); break;
    case 8: pick<8>(ph, k); break;
    default: *k = KernelSet{};
    }
}

const void *dgk_vol_fixed_3d_f32(int order, int phys, int C, int NT, int forced, int batched)
{
    return find_fixed_vol<3, 1, float>(order, phys, C, NT, forced, batched, std::make_index_sequence<kNumTiles>{});
}

const void *dgk_face_fixed_3d_f32(int order, int phys, int C, int NT, int batched)
{
    return find_fixed_face<3, 1, float>(order, phys, C, NT, batched, std::make_index_sequence<kNumTiles>{});
}

int dgk_upload_3d_f32(const Tab<double> *d, const Tab<float> *f)
{
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabd), d, sizeof(Tab<double>) * (MAXP + 1)) != hipSuccess) return -1;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabf), f, sizeof(Tab<float>) * (MAXP + 1)) != hipSuccess) return -1;
    return 0;
}

}  // namespace dgk
