// Rigid-translation gradient of the relative binding energy: the complex
// surface's vertices owned by the ligand (the atom minimising
// |v - r_a| - R_a is a ligand atom) and the sum of the ligand's site and
// vertex gradients.
#include "kernels.hpp"

namespace pbmp {

namespace {

__global__ void k_vertex_owner(int nv, int m, int first_ligand, const double *__restrict__ verts,
                               const double *__restrict__ xyz, const double *__restrict__ radii,
                               int *__restrict__ owner) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double p[3] = {verts[3 * v], verts[3 * v + 1], verts[3 * v + 2]};
  double best = 0.0;
  int ab = -1;
  for (int a = 0; a < m; ++a) {
    const double dx = p[0] - xyz[3 * a], dy = p[1] - xyz[3 * a + 1], dz = p[2] - xyz[3 * a + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz) - radii[a];
    if (ab < 0 || d < best) {  // ties: the lower atom index
      best = d;
      ab = a;
    }
  }
  owner[v] = ab >= first_ligand ? 1 : 0;
}

// one block: fixed-order sums over the ligand's sites and owned vertices
constexpr int kSumThreads = 256;
__global__ __launch_bounds__(kSumThreads) void k_translation_sum(
    int nv, int m, int first_ligand, const int *__restrict__ owner,
    const double *__restrict__ g_verts, const double *__restrict__ g_xyz,
    double *__restrict__ out) {
  __shared__ double red[4][kSumThreads];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int v = threadIdx.x; v < nv; v += kSumThreads)
    if (owner[v]) {
      for (int c = 0; c < 3; ++c) acc[c] += g_verts[3 * v + c];
      acc[3] += 1.0;
    }
  for (int a = first_ligand + threadIdx.x; a < m; a += kSumThreads)
    for (int c = 0; c < 3; ++c) acc[c] += g_xyz[3 * a + c];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

void launch_translation_sum(hipStream_t s, int nv, int m, int first_ligand,
                            const double *verts, const double *xyz, const double *radii,
                            const double *g_verts, const double *g_xyz, int *owner,
                            double *out) {
  if (nv > 0)
    hipLaunchKernelGGL(k_vertex_owner, dim3((nv + 255) / 256), dim3(256), 0, s, nv, m,
                       first_ligand, verts, xyz, radii, owner);
  hipLaunchKernelGGL(k_translation_sum, dim3(1), dim3(kSumThreads), 0, s, nv, m, first_ligand,
                     owner, g_verts, g_xyz, out);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
