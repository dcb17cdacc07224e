// Work memory for the entry point that allocates nothing
// (pbmp_site_fields_noalloc): one file-scope device array per GPU, whose
// device address is looked up once per device with hipGetSymbolAddress and
// kept; host code uses that address, never the array's name.
#include <mutex>

#include "kernels.hpp"
#include "runtime.hpp"

namespace pbmp {

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kScratchBytes; }

double *static_scratch() {
  int dev = 0;
  PBMP_HIP(hipGetDevice(&dev));
  PBMP_REQUIRE(dev >= 0 && dev < kMaxDevices, PBMP_EARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    PBMP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PBMP_REQUIRE(p != nullptr, PBMP_EHIP, "no device address for the static scratch");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  return g_scratch_ptr[dev];
}

// pbmp_site_fields into the static scratch: the density permuted into the
// internal panel order, then the per-chunk partial sums of the readout.
void Runtime::site_fields_noalloc(const double *x, double *out) {
  PBMP_REQUIRE(N_ > 0 && M_ > 0, PBMP_ESTATE, "no mesh or sites");
  PBMP_REQUIRE(x != nullptr && out != nullptr, PBMP_EARG, "null input or output");
  PBMP_REQUIRE(!outer_, PBMP_ESTATE, "not available with a Stern layer");
  const size_t cap = kScratchBytes / sizeof(double);
  const size_t nx = 2 * (size_t)N_, per_chunk = 10 * (size_t)M_;
  PBMP_REQUIRE(nx + per_chunk <= cap, PBMP_EARG,
               "mesh and sites need more than the 32 MiB static scratch "
               "(2 nt + 10 m doubles at least)");
  const int nchunk = (int)std::min<size_t>((size_t)ro_chunks_, (cap - nx) / per_chunk);
  double *scr = static_scratch();
  double *xi = scr, *part = scr + nx;
  launch_permute(s_, N_, 2, d_perm_.p, x, xi, true);
  launch_pack_strengths(s_, N_, ru_.nf, geo_.p, xi, src64_.p, src32_.p);
  launch_readout(s_, fp64(), true, N_, M_, src64_.p, src32_.p, geo_.p, verts_.p, tri_.p, ru_,
                 xi, sxyz_.p, srow_.p, scol_.p, nchunk, part, out);
  sync();
}

}  // namespace pbmp
