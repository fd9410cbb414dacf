// Velocity-Verlet NVE driver on the device (a test harness for the potential, not
// part of one step): x, v stay in float64 on the device, forces come from the
// library's step (neighbour lists reused with a skin when dp_set_skin is on), and
// the potential and kinetic energies of every step are returned for the drift.
//   v += dt/2 F/m;  x += dt v;  F = F(x);  v += dt/2 F/m     (units A, fs, amu, eV)
#include <vector>

#include "../../include/dp.h"
#include "dp_internal.h"

namespace dp {
namespace {

constexpr double ACC = 9.648533e-3;  // 1 eV/(A amu) in A/fs^2

__global__ void k_kick(double *__restrict__ v, const double *__restrict__ F, const int *__restrict__ types,
                       const double *__restrict__ inv_m, int n, double h) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  v[k] += h * F[k] * inv_m[types[k / 3]];
}

__global__ void k_drift(double *__restrict__ x, const double *__restrict__ v, int n, double dt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 3 * n) x[k] += dt * v[k];
}

__global__ void k_kinetic(const double *__restrict__ v, const int *__restrict__ types,
                          const double *__restrict__ mass, int n, double *__restrict__ ke) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
  ke[i] = 0.5 * mass[types[i]] * (vx * vx + vy * vy + vz * vz) / ACC;
}

}  // namespace
}  // namespace dp

using namespace dp;

extern "C" int dp_nve_run(dp_model *m, int64_t natoms, double *d_coords, double *d_vel, const int32_t *d_types,
                          const double *masses, const double *box, double dt_fs, int nsteps, double *epot,
                          double *ekin, void *hip_stream) {
  if (!m || natoms < 1 || !d_coords || !d_vel || !d_types || !masses || nsteps < 0 || !(dt_fs > 0.0)) {
    set_error("dp_nve_run: bad argument");
    return DP_ERR_ARG;
  }
  for (int t = 0; t < m->ntypes; ++t)
    if (!(masses[t] > 0.0)) {
      set_error("dp_nve_run: masses must be positive");
      return DP_ERR_ARG;
    }
  if (hipSetDevice(m->device) != hipSuccess) return DP_ERR_HIP;
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = (int)natoms;
  double *F = nullptr, *E = nullptr, *ke = nullptr, *kesum = nullptr, *mass = nullptr, *inv_m = nullptr;
  auto cleanup = [&]() {
    void *ps[] = {F, E, ke, kesum, mass, inv_m};
    for (void *p : ps)
      if (p) (void)hipFree(p);
  };
  std::vector<double> hm(masses, masses + m->ntypes), him(m->ntypes);
  for (int t = 0; t < m->ntypes; ++t) him[t] = ACC / hm[t];
  if (hipMalloc(&F, 3 * natoms * sizeof(double)) != hipSuccess || hipMalloc(&E, sizeof(double)) != hipSuccess ||
      hipMalloc(&ke, natoms * sizeof(double)) != hipSuccess || hipMalloc(&kesum, sizeof(double)) != hipSuccess ||
      hipMalloc(&mass, m->ntypes * sizeof(double)) != hipSuccess ||
      hipMalloc(&inv_m, m->ntypes * sizeof(double)) != hipSuccess ||
      hipMemcpy(mass, hm.data(), m->ntypes * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(inv_m, him.data(), m->ntypes * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    set_error("dp_nve_run: allocation failed");
    return DP_ERR_OOM;
  }
  const dim3 b3((3 * n + 255) / 256), b1((n + 255) / 256), th(256);
  int worst = DP_OK;
  auto energies = [&](int step) -> int {
    hipLaunchKernelGGL(k_kinetic, b1, th, 0, st, d_vel, d_types, mass, n, ke);
    launch_sum(m->ws, ke, kesum, st);
    double e = 0.0, k = 0.0;
    if (hipMemcpyAsync(&e, E, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&k, kesum, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("dp_nve_run: copy failed");
      return DP_ERR_HIP;
    }
    if (epot) epot[step] = e;
    if (ekin) ekin[step] = k;
    return DP_OK;
  };
  int s = dp_compute_device(m, natoms, d_coords, d_types, box, E, F, nullptr, nullptr, st);
  if (s > worst) worst = s;
  if (s >= 0) s = energies(0);
  for (int step = 1; s >= 0 && step <= nsteps; ++step) {
    hipLaunchKernelGGL(k_kick, b3, th, 0, st, d_vel, F, d_types, inv_m, n, 0.5 * dt_fs);
    hipLaunchKernelGGL(k_drift, b3, th, 0, st, d_coords, d_vel, n, dt_fs);
    s = dp_compute_device(m, natoms, d_coords, d_types, box, E, F, nullptr, nullptr, st);
    if (s < 0) break;
    if (s > worst) worst = s;
    hipLaunchKernelGGL(k_kick, b3, th, 0, st, d_vel, F, d_types, inv_m, n, 0.5 * dt_fs);
    s = energies(step);
  }
  (void)hipStreamSynchronize(st);
  cleanup();
  return s < 0 ? s : worst;
}
