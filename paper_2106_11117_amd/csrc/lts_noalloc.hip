// Forward solve that allocates no device memory (lts_forward_noalloc).
//
// Its device scratch (the sorted per-sample tables, the staging flag and the
// two time levels of the state) lives in one file-scope device array per GPU,
// `scratch`, of fixed size.  The array's device address is taken once per
// device at context creation (hipGetSymbolAddress with that device current)
// and kept in a per-device table; host code uses only that address, never the
// array's name.  Every call on a device shares the device's array and leaves
// its last contents: everything a solve reads is written by that solve first
// (the staged tables by the upload, both state buffers in full by the initial
// state kernel, the flag by a fill kernel), and two calls that overlap on one
// GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ctx.h"

namespace lts {

namespace {

constexpr size_t kScratchBytes = LTS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

size_t a256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// Called by lts_create with `device` current.
lts_status noalloc_attach(lts_ctx c, int device) {
  if (device < 0 || device >= kMaxDevices) return arg_fail(c, "device ordinal too large for the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return hip_fail(c, hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = p;
  }
  return LTS_OK;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch[device] : nullptr;
}

}  // namespace lts

using namespace lts;

extern "C" lts_status lts_forward_noalloc(lts_ctx c, int32_t level, const lts_samples* S, int32_t precision,
                                          double* Q_out) {
  if (!c) return LTS_ERR_ARG;
  c->err.clear();
  if (level < 0 || level >= (int32_t)c->levels.size()) return arg_fail(c, "no such level");
  const DevLevel& lv = *c->levels[level];
  if (precision != LTS_FP64 && precision != LTS_FP32_STEP) return arg_fail(c, "bad precision");
  if (S && S->n > 0 && !Q_out) return arg_fail(c, "Q_out is NULL");
  // the scratch a batch of n samples needs (checked before anything is read)
  const size_t n = S && S->n > 0 ? (size_t)S->n : 0;
  const size_t es = precision == LTS_FP32_STEP ? sizeof(float) : sizeof(double);
  const size_t o_perm = 256, o_ns = o_perm + a256(n * 4), o_k = o_ns + a256(n * 4);
  const size_t o_x = o_k + a256(n * lv.H.n_blocks * 8), o_c = o_x + a256(n * 16);
  const size_t o_q = o_c + a256(n * (lv.H.p + 1) * 8), o_b0 = o_q + a256(n * 8);
  const size_t sb = a256(n * lv.nodes * es), need = o_b0 + 2 * sb;
  if (need > kScratchBytes)
    return arg_fail(c, "the batch needs " + std::to_string(need) + " bytes of device scratch; the no-allocation "
                       "scratch holds " + std::to_string(kScratchBytes) + " (fewer samples per call)");
  Staged st;
  lts_status r = stage_samples(c, lv, S, st);
  if (r != LTS_OK) return r;
  if (st.n == 0) return LTS_OK;
  LTS_HIP(c, hipSetDevice(c->device));
  char* base = static_cast<char*>(scratch_of(c->device));
  if (!base) {
    c->err = "no-allocation scratch not attached on this device";
    return LTS_ERR_STATE;
  }
  const StagedDev d{(double*)(base + o_k), (double*)(base + o_x), (double*)(base + o_c), (int*)(base + o_ns),
                    (int*)(base + o_perm), (int*)base};
  if ((r = upload_staged(c, lv, st, S, d)) != LTS_OK) return r;
  double* dQ = (double*)(base + o_q);
  r = forward_device_states(c, lv, st.n, d.kappa, d.coef, d.nsteps, d.x0, S->width, st.nsteps, precision, false, dQ,
                            (double*)(base + o_b0), (double*)(base + o_b0 + sb), false);
  if (r != LTS_OK) return r;
  return finish_Q(c, st, dQ, d, Q_out);
}
