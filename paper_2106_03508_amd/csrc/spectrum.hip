// Broadened spectral function of the dressed Green's function in the
// physical space (the simulated photoelectron spectra of the application
// section, broadening factor eta):
//   A(w) = -1/pi Im Tr[P G(w + i eta)] = eta/pi sum_l w_l / ((w - lam_l)^2 + eta^2),
//   w_l  = sum_p P_p u[p][l]^2,
// G being the physical block of the resolvent of the extended Hamiltonian
// whose eigenpairs are the poles (lam_l, u[:, l]).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "agf2_internal.h"

namespace agf2 {

namespace {

constexpr int ST = 256;

constexpr int PS = 16;   // row ranges of the pole-weight sums

// Device scratch of the allocation-free entry point: the PS partial
// pole-weight rows and the summed weights, [(PS + 1) * kNoallocMaxPole]
// doubles (4.25 MiB), one copy per GPU for the life of the process. Host code
// must not use the name of this array as an address: it takes the per-device
// address that hipGetSymbolAddress returns (noalloc_scratch below).
constexpr int kNoallocMaxPole = AGF2_SPECTRUM_NOALLOC_MAX_POLE;
static __device__ __align__(256) double scratch[(PS + 1) * kNoallocMaxPole];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

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

namespace {

// the three launches over a caller-provided scratch of (PS + 1) * npole doubles
void spectral_launch(hipStream_t st, int nphys, int npole, const double* e_pole,
                     const double* u_pole, const double* weight, int nomega,
                     const double* omega, double eta, double* A, double* part) {
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

}  // namespace

void spectral_function(Handle& h, int nphys, int npole, const double* e_pole,
                       const double* u_pole, const double* weight, int nomega,
                       const double* omega, double eta, double* A) {
  if (nomega == 0) return;
  ProfScope ps(h, "spectrum", 3.0 * nphys * (double)npole + 5.0 * nomega * (double)npole,
               8.0 * ((double)nphys * npole + 2.0 * npole + 2.0 * nomega));
  double* part = h.ws_spec.as<double>((long)(PS + 1) * npole);
  spectral_launch(h.stream, nphys, npole, e_pole, u_pole, weight, nomega, omega, eta, A, part);
}

// Device address of this GPU's scratch array: resolved once per device with
// that device current (the handle's set-up calls this), then cached.
double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw Error{AGF2_ERR_ARG, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    DeviceGuard g(device);
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{AGF2_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e)};
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

// The same launches on the device's scratch array: no allocation, no event,
// no host synchronisation.
void spectral_function_noalloc(Handle& h, int nphys, int npole, const double* e_pole,
                               const double* u_pole, const double* weight, int nomega,
                               const double* omega, double eta, double* A) {
  if (npole > kNoallocMaxPole)
    throw Error{AGF2_ERR_ARG, "npole exceeds AGF2_SPECTRUM_NOALLOC_MAX_POLE (" +
                                  std::to_string(kNoallocMaxPole) + ")"};
  if (nomega == 0) return;
  spectral_launch(h.stream, nphys, npole, e_pole, u_pole, weight, nomega, omega, eta, A,
                  noalloc_scratch(h.device));
}

}  // namespace agf2
