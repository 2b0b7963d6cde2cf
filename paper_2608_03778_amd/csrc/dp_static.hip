// dp_forward_static: a modeled (or frozen-beta) forward of one query that
// allocates nothing.  Its intermediate arrays live in one file-scope device
// array, `scratch`, of a fixed size; each GPU the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name
// to a kernel (in host code that name is a host-side stand-in, not a device
// address): the device address of each GPU's copy is resolved once, when a
// context is created on that GPU, and kept here.
#include <mutex>

#include "dp_internal.h"

namespace {

// Scratch layout for a design of n nets (one query column), every part
// 256-byte aligned:
//   SP (stored form)      float  [n]      4 n bytes
//   capacitance           float  [n]      4 n bytes (internal numbering)
//   frozen beta           float  [n]      4 n bytes (internal numbering)
//   power partial sums    double [chunks]
constexpr int64_t kMaxNets = int64_t(1) << 21;
constexpr int64_t kPartBytes = 64 << 10;  // >= 8 * power_partial_doubles(kMaxNets, 1, 0, 0)
constexpr int64_t kScratchBytes = 12 * kMaxNets + kPartBytes + 3 * 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` on each GPU (null = not resolved)

int64_t up256(int64_t b) { return (b + 255) & ~int64_t(255); }

}  // namespace

namespace dp {

dp_status static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(DP_E_UNSUPPORTED, "static scratch: device id beyond " + std::to_string(kMaxDevices));
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return DP_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(DP_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                              hipGetErrorString(e));
  g_ptr[device] = p;
  return DP_OK;
}

}  // namespace dp

extern "C" dp_status dp_forward_static(const dp_design *d, const dp_params *prm,
                                       const float *pi_prob, const float *cap, const float *beta,
                                       float *power, float *sp, float *tr) {
  using dp::fail;
  if (!d || !prm || !pi_prob || !cap || !power)
    return fail(DP_E_INVALID, "dp_forward_static: NULL argument");
  DP_TRY(dp::params_ok(prm));
  if (prm->mode == DP_HYBRID)
    return fail(DP_E_UNSUPPORTED,
                "dp_forward_static: DP_HYBRID needs simulation words; use dp_forward");
  if ((prm->mode == DP_FROZEN_BETA) != (beta != nullptr))
    return fail(DP_E_INVALID, "dp_forward_static: beta is required in DP_FROZEN_BETA and only there");
  if ((int64_t)d->n_nets > kMaxNets)
    return fail(DP_E_INVALID, "dp_forward_static: the design has " + std::to_string(d->n_nets) +
                                  " nets; the static scratch holds at most " +
                                  std::to_string(kMaxNets));
  const int device = d->ctx->device;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
  }
  if (!base) return fail(DP_E_STATE, "dp_forward_static: the static scratch of this device is not set up");
  DP_HIP_TRY(hipSetDevice(device));
  const int32_t nn = d->n_nets;
  char *s0 = static_cast<char *>(base);
  float *spp = reinterpret_cast<float *>(s0);
  float *capi = reinterpret_cast<float *>(s0 + up256(4 * (int64_t)nn));
  float *betai = reinterpret_cast<float *>(reinterpret_cast<char *>(capi) + up256(4 * (int64_t)nn));
  double *part = reinterpret_cast<double *>(reinterpret_cast<char *>(betai) + up256(4 * (int64_t)nn));
  if ((int64_t)dp::power_partial_doubles(nn, 1, 0, 0) * 8 > kPartBytes)
    return fail(DP_E_INVALID, "dp_forward_static: power partials exceed the static scratch");

  hipStream_t s = d->ctx->stream;
  const dp::GraphView g = dp::design_view(d);
  const int32_t *i2e = d->int2ext.as<int32_t>();
  DP_HIP_TRY(dp::launch_load_pi(pi_prob, spp, d->n_pi, 1, s));
  DP_HIP_TRY(dp::launch_gather_nets_f32(cap, i2e, capi, nn, s));
  if (beta) DP_HIP_TRY(dp::launch_gather_nets_f32(beta, i2e, betai, nn, s));
  for (int32_t l = 1; l <= d->depth;) {
    if (dp::pairs_levels(d, l, 1)) {  // levels l and l + 1 in one launch
      const int32_t a0 = d->level_ptr[l], a1 = d->level_ptr[l + 1], b1 = d->level_ptr[l + 2];
      DP_HIP_TRY(dp::launch_sp_pair(g, dp::SpLevel{spp, 1, a0, a1 - a0},
                                    dp::SpLevel{spp, 1, a1, b1 - a1}, s));
      l += 2;
      continue;
    }
    DP_TRY(dp::for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
      DP_HIP_TRY(dp::launch_sp_level(g, dp::SpLevel{spp, 1, g0, n}, cells, s));
      return DP_OK;
    }));
    ++l;
  }
  dp::PowerArgs pa{};
  pa.sp = spp;
  pa.beta_frozen = beta ? betai : nullptr;
  pa.beta_shared = 1;
  pa.cap = capi;
  pa.kappa = (float)dp::kappa(*prm);
  pa.beta_min = (float)prm->beta_min;
  pa.beta_max = (float)prm->beta_max;
  pa.mode = prm->mode;
  pa.n_pi = d->n_pi;
  pa.n_nets = nn;
  pa.G = d->n_gates;
  pa.B = 1;
  pa.partial = part;
  pa.n_chunks = dp::power_chunks(nn);
  pa.power = power;
  DP_HIP_TRY(dp::launch_power(pa, s));
  if (sp || tr) {
    dp::ExportArgs ea{};
    ea.sp = spp;
    ea.int2ext = i2e;
    ea.o_sp = sp;
    ea.o_tr = tr;
    ea.n_nets = nn;
    ea.B = 1;
    DP_HIP_TRY(dp::launch_export(ea, s));
  }
  return DP_OK;
}
