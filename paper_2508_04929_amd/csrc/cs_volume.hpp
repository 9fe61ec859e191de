// Voxelisation and FSC kernels (k_volume.hip).
#pragma once

#include "cs_internal.hpp"

namespace cs {

struct VoxGeom {
  int N;        // Gaussians
  int D;        // voxels per side (a multiple of 8)
  int c0;       // D / 2: the grid origin
  int nb;       // bricks per side, D / 8
  float pixel;  // Angstrom per voxel
  float q_cut;  // truncation of the squared Mahalanobis distance
};

__global__ void k_vox_prep(const float4 *gc, VoxGeom V, float4 *rec, int4 *box, double *wpart);
__global__ void k_vox_count(const int4 *box, VoxGeom V, int *count);
__global__ void k_vox_scan(const int *count, int nbr, const double *wpart, int nwp, int *off,
                           double *scale);
__global__ void k_vox_fill(const int4 *box, VoxGeom V, const int *off, int *cursor, int *list);
__global__ void k_vox_eval(const float4 *rec, const int *list, const int *off, VoxGeom V,
                           const double *scale, float *vol);
constexpr int kEnergyBlocks = 1024;  // fixed grid of the energy pass (order-stable sums)
__global__ void k_fsc_energy_part(const float *va, const float *vb, int64_t n, double *part);
__global__ void k_fsc_energy_scale(const double *part, int D, double *scale);
__global__ void k_fsc_shells(const float2 *fa, const float2 *fb, int D, const double *scale,
                             unsigned long long *sums);
__global__ void k_fsc_final(const unsigned long long *sums, int ns, const double *scale,
                            float *fsc);
__global__ void k_fsc_resolution(const float *fsc, int ns, int D, float pixel, float threshold,
                                 int *shell, float *resolution);
__global__ void k_fill_u64z(unsigned long long *p, int n);
__global__ void k_fill_i32z(int *p, int n);

}  // namespace cs
