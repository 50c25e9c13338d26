// dg_registry.hpp -- host-side handles of the kernel instantiations.
#pragma once
#include <stddef.h>

#include "dg_common.hpp"

namespace dgk {

// Kernels and LDS-size functions of one (dim, order, precision, physics)
// instantiation; physics PH = 0 Euler, 1 Navier-Stokes, 2 artificial
// viscosity, 3 Navier-Stokes with the tracer, 4..7 the same on the
// total-degree basis.  The function pointers are the host stubs of
// __global__ functions, launched with hipLaunchKernel.
struct KernelSet {
    const void *vol;
    const void *face;
    const void *cfl;   // FP64 units only
    const void *vol_b;     // grouped (batched ensemble) variants
    const void *face_b;
    const void *cfl_b;     // FP64 units only
    size_t (*vol_lds)(int C, int NU);   // NU: point-value arrays per cell (the stored fields)
    size_t (*face_lds)(int C);
    size_t (*cfl_lds)(int C, int nt);
    const void *limit;     // positivity limiter (FP64 units only)
    size_t (*limit_lds)(int C, int nt);
    const void *fpts;      // driving field -> Gauss-point values (256 threads, grid: arrays / FA)
};

void dgk_get_2d_f64(int P, int ph, KernelSet *k);
void dgk_get_3d_f64(int P, int ph, KernelSet *k);
void dgk_get_2d_f32(int P, int ph, KernelSet *k);
void dgk_get_3d_f32(int P, int ph, KernelSet *k);
// Fixed-tile volume kernel for (order, physics, cells per block, threads,
// forcing) if the tuned table has one for this unit, else null; batched = 1
// selects the grouped (ensemble) variant.
const void *dgk_vol_fixed_2d_f64(int order, int phys, int C, int NT, int forced, int batched);
const void *dgk_vol_fixed_3d_f64(int order, int phys, int C, int NT, int forced, int batched);
const void *dgk_vol_fixed_2d_f32(int order, int phys, int C, int NT, int forced, int batched);
const void *dgk_vol_fixed_3d_f32(int order, int phys, int C, int NT, int forced, int batched);
// Fixed-tile face kernel for (order, physics, faces per pencil, threads).
const void *dgk_face_fixed_2d_f64(int order, int phys, int C, int NT, int batched);
const void *dgk_face_fixed_3d_f64(int order, int phys, int C, int NT, int batched);
const void *dgk_face_fixed_2d_f32(int order, int phys, int C, int NT, int batched);
const void *dgk_face_fixed_3d_f32(int order, int phys, int C, int NT, int batched);
int dgk_upload_2d_f64(const Tab<double> *d, const Tab<float> *f);
int dgk_upload_3d_f64(const Tab<double> *d, const Tab<float> *f);
int dgk_upload_2d_f32(const Tab<double> *d, const Tab<float> *f);
int dgk_upload_3d_f32(const Tab<double> *d, const Tab<float> *f);

}  // namespace dgk
