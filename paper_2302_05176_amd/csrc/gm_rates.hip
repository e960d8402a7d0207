// gm_rates.hip -- issue-rate probes for the roofline of the sketch kernels.
//
// Each lane draws `steps` arrivals (or plain keys) of one synthetic element
// (index = lane) exactly as the sketch kernels do -- the draw specification
// of gm_draw.h, the Renyi prefix O_z = fma(E_z, 1/(k-z+1), O_{z-1}) of
// Eq. (7)-(8), the Fisher-Yates target -- with no memory traffic besides one
// result per lane.  The achieved rate is the best the VALU sustains for the
// method's per-arrival arithmetic, the reference the sketch kernels' achieved
// fraction is read against.
#include "gm_common.h"

namespace gm {

__global__ __launch_bounds__(256) void arrival_rate_kernel(int64_t lanes, int32_t k,
                                                           uint64_t seed_mix, double* out) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= lanes) return;
  const uint64_t P = mix(seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(g)));
  const double r = 1.0 / (1.0 + static_cast<double>(g & 7));
  double O = 0.0, acc = 0.0;
  for (int32_t z = 1; z <= k; ++z) {
    const double E = exp1(draw(P, kTagArrival, static_cast<uint32_t>(z)));
    O = fma(E, 1.0 / static_cast<double>(k - z + 1), O);
    const int32_t j = randint(draw(P, kTagShuffle, static_cast<uint32_t>(z)), z, k);
    acc += O * r + static_cast<double>(j);
  }
  out[g] = acc;
}

__global__ __launch_bounds__(256) void key_rate_kernel(int64_t lanes, int32_t k,
                                                       uint64_t seed_mix, double* out) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= lanes) return;
  const uint64_t P = mix(seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(g)));
  const double r = 1.0 / (1.0 + static_cast<double>(g & 7));
  double best = bitsd(kInfBits);
  for (int32_t j = 0; j < k; ++j) {
    const double t = exp1(draw(P, kTagPlain, static_cast<uint32_t>(j))) * r;
    best = t < best ? t : best;
  }
  out[g] = best;
}

hipError_t launch_rate_probe(int what, int64_t lanes, int32_t steps, uint64_t seed_mix,
                             double* out, hipStream_t stream) {
  const int64_t grid = (lanes + 255) / 256;
  if (what == 0)
    hipLaunchKernelGGL(arrival_rate_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                       stream, lanes, steps, seed_mix, out);
  else
    hipLaunchKernelGGL(key_rate_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream,
                       lanes, steps, seed_mix, out);
  return hipGetLastError();
}

}  // namespace gm
