// Broadened spectral function of the dressed Green's function in the
// physical space (the simulated photoelectron spectra of the application
// section, broadening factor eta):
//   A(w) = -1/pi Im Tr[P G(w + i eta)] = eta/pi sum_l w_l / ((w - lam_l)^2 + eta^2),
//   w_l  = sum_p P_p u[p][l]^2,
// G being the physical block of the resolvent of the extended Hamiltonian
// whose eigenpairs are the poles (lam_l, u[:, l]).
#include <algorithm>
#include <cmath>

#include "agf2_internal.h"

namespace agf2 {

namespace {

constexpr int ST = 256;

constexpr int PS = 16;   // row ranges of the pole-weight sums

// part[y][l] = sum over rows p of range y of P_p u[p][l]^2 (P = 1 when weight
// is NULL); threads over poles, so each read of a row of u is contiguous
// across the wave
__global__ __launch_bounds__(ST) void pole_weight_kernel(int nphys, int npole, const double* u,
                                                         const double* weight, double* part) {
  const int l = blockIdx.x * ST + threadIdx.x;
  if (l >= npole) return;
  const int per = (nphys + PS - 1) / PS;
  const int p0 = blockIdx.y * per, p1 = min(nphys, p0 + per);
  double s = 0.0;
  for (int p = p0; p < p1; ++p) {
    const double x = u[(long)p * npole + l];
    s += (weight ? weight[p] : 1.0) * x * x;
  }
  part[(long)blockIdx.y * npole + l] = s;
}

// w[l] = sum_y part[y][l] in ascending y
__global__ __launch_bounds__(ST) void pole_weight_sum_kernel(int npole, const double* part,
                                                             double* w) {
  const int l = blockIdx.x * ST + threadIdx.x;
  if (l >= npole) return;
  double s = 0.0;
  for (int y = 0; y < PS; ++y) s += part[(long)y * npole + l];
  w[l] = s;
}

// A[k] = eta/pi sum_l w[l] / ((omega[k] - lam[l])^2 + eta^2): one wave per
// frequency (four per workgroup), lane j summing poles j, j + 64, ... in
// ascending order, then a fixed shuffle tree across the wave
__global__ __launch_bounds__(ST) void spectral_kernel(int npole, const double* lam,
                                                      const double* w, int nomega,
                                                      const double* omega, double eta,
                                                      double* A) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (ST / 64) + (threadIdx.x >> 6);
  if (k >= nomega) return;   // uniform over the wave
  const double om = omega[k];
  const double eta2 = eta * eta;
  double acc = 0.0;
  for (int l = lane; l < npole; l += 64) {
    const double d = om - lam[l];
    acc += w[l] / (d * d + eta2);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) A[k] = acc * (eta / M_PI);
}

}  // namespace

void spectral_function(Handle& h, int nphys, int npole, const double* e_pole,
                       const double* u_pole, const double* weight, int nomega,
                       const double* omega, double eta, double* A) {
  if (nomega == 0) return;
  hipStream_t st = h.stream;
  ProfScope ps(h, "spectrum", 3.0 * nphys * (double)npole + 5.0 * nomega * (double)npole,
               8.0 * ((double)nphys * npole + 2.0 * npole + 2.0 * nomega));
  double* part = h.ws_spec.as<double>((long)(PS + 1) * npole);
  double* w = part + (long)PS * npole;
  const int gl = (npole + ST - 1) / ST;
  hipLaunchKernelGGL(pole_weight_kernel, dim3(gl, PS), dim3(ST), 0, st, nphys, npole, u_pole,
                     weight, part);
  AGF2_CHECK_LAUNCH();
  hipLaunchKernelGGL(pole_weight_sum_kernel, dim3(gl), dim3(ST), 0, st, npole, part, w);
  AGF2_CHECK_LAUNCH();
  const int per = ST / 64;
  hipLaunchKernelGGL(spectral_kernel, dim3((nomega + per - 1) / per), dim3(ST), 0, st, npole,
                     e_pole, w, nomega, omega, eta, A);
  AGF2_CHECK_LAUNCH();
}

}  // namespace agf2
