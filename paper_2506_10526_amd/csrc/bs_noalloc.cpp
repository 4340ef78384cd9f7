// Entry points that allocate nothing: for callers that cannot call hipMalloc (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// Their scratch memory is a file-scope device array of fixed size.  In host code the array's
// name is only a host-side stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress (from bs_create, with that device current) and that pointer is what the
// kernels receive.  Every call on a device shares that device's array: calls that overlap on
// one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "bs_ctx.h"
#include "bs_kernels.h"

namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;   // 8 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the scratch array (once per device; `device` must be current).
int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return BS_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return BS_EHIP;
  }
  g_ptr[device] = p;
  return BS_OK;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

// Monopole B(k1, mu, t) of a cylindrical 3D bispectrum (Sec. 2.2 Eq. shape, Sec. 5), as
// bs_monopole, with the per-block partial bins in the scratch array.
extern "C" int bs_monopole_noalloc(bs_ctx* c, int32_t nc, int32_t n_tri, const double* kperp, double kpar_unit,
                                   const void* Bcyl, int32_t n_k1, const double* k1_edges, double* mean,
                                   int64_t* count) {
  if (!c) return BS_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return ctx_fail(c, BS_EHIP, "hipSetDevice");
  if (nc < 1 || nc > 65536) return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: nc must be in [1, 65536]");
  if (n_tri < 0 || (long long)n_tri * nc > (1LL << 31) - 1)
    return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: n_tri * nc must be in [0, 2^31)");
  if (n_k1 < 1 || n_k1 > MONO_MAX_K1) return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: n_k1 must be in [1, 64]");
  if (!(kpar_unit > 0.0) || !std::isfinite(kpar_unit))
    return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: kpar_unit must be > 0");
  if (!k1_edges || !mean || !count || (n_tri > 0 && (!kperp || !Bcyl)))
    return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: NULL pointer");
  unsigned char* base = static_cast<unsigned char*>(scratch_of(c->device));
  if (!base) return ctx_fail(c, BS_EHIP, "bs_monopole_noalloc: scratch address of this device unknown");
  const int nb = n_k1 * 25;
  // a wave per row, blocks of four rows, at most 2048 blocks (as bs_monopole) and at most as many as the
  // scratch holds
  const long long rows = (long long)n_tri * nc;
  // per block: its partial sums and counts (12 B a bin) and 1 / PART_KC of a group's sums and counts (16 B)
  const long long per_block = (long long)nb * 13;
  const long long cap = (long long)(kScratchBytes - 1024) / per_block;
  const int nblocks = (int)std::max(1LL, std::min(std::min(2048LL, cap), (rows + 3) / 4));
  const int groups = part_groups(nblocks);
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t sum_bytes = up((size_t)nblocks * nb * sizeof(double));
  const size_t cnt_bytes = up((size_t)nblocks * nb * sizeof(int));
  const size_t gs_bytes = up((size_t)groups * nb * sizeof(double));
  if (sum_bytes + cnt_bytes + gs_bytes + (size_t)groups * nb * sizeof(long long) > kScratchBytes)
    return ctx_fail(c, BS_EINVAL, "bs_monopole_noalloc: partial bins exceed the scratch array");
  MonoArgs a{};
  a.B = static_cast<const double*>(Bcyl);
  a.kperp = kperp;
  a.k1e = k1_edges;
  a.psum = reinterpret_cast<double*>(base);            // every block and group stores all of its
  a.pcnt = reinterpret_cast<int*>(base + sum_bytes);   // slots: nothing needs to start at zero
  a.stage_s = reinterpret_cast<double*>(base + sum_bytes + cnt_bytes);
  a.stage_c = reinterpret_cast<long long*>(base + sum_bytes + cnt_bytes + gs_bytes);
  a.kpar_unit = kpar_unit;
  a.nc = nc;
  a.nt = n_tri;
  a.nk = n_k1;
  launch_mono_bin(a, nblocks, c->stream);
  launch_mono_fin(a, nblocks, mean, count, c->stream);
  if (hipGetLastError() != hipSuccess) return ctx_fail(c, BS_EHIP, "bs_monopole_noalloc launch");
  return BS_OK;
}
