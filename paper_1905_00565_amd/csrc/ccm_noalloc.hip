// ccm_noalloc.hip -- ccm_dev_noalloc: the cross map of ccm_dev with every
// device buffer of the call taken from one static workspace per device, for
// callers that cannot allocate device memory.
//
// The workspace is a file-scope device array; in host code its name only
// stands for the symbol, so its device address on each device is looked up
// once (with that device current, at context creation) and every host-side
// use goes through that address.  Every call on a device shares the
// device's workspace: calls that overlap on one device race.
#include "ccm_context.h"

namespace {

constexpr uint64_t kWorkspaceBytes = CCM_NOALLOC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kWorkspaceBytes];

std::mutex g_mu;
char* g_base[kMaxDevices] = {};   // device address of the workspace, per device

char* workspace(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device >= 0 && device < kMaxDevices ? g_base[device] : nullptr;
}

uint64_t up256(uint64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

namespace ccmh {

bool noalloc_setup(int device, std::string* err) {
  if (device < 0 || device >= kMaxDevices) {
    *err = "device index beyond the workspace table";
    return false;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_base[device]) return true;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    *err = std::string("workspace address: ") + hipGetErrorString(e);
    return false;
  }
  g_base[device] = static_cast<char*>(ptr);
  return true;
}

}  // namespace ccmh

using namespace ccmh;

extern "C" ccm_status ccm_dev_noalloc(ccm_ctx* c, const double* X, const double* Y, int64_t N,
                                      int32_t E, int32_t tau, const int64_t* L, int32_t nL,
                                      int32_t r, uint64_t seed, const ccm_opts* opts,
                                      double* rho_xy, double* rho_yx, int64_t* L_eff,
                                      void* stream) {
  return guarded(c, [&] {
    if (!X || !Y || !rho_xy || !rho_yx) fail(CCM_E_INVAL, "NULL device pointer");
    Spec s = make_spec(N, &E, 1, &tau, 1, L, nL, r, seed, opts);
    if (s.flags & ~CCM_FLAG_NO_GRAPH)
      fail(CCM_E_INVAL, "the no-allocation form runs the default batched launches only");
    s.flags = 0;
    s.wave_limit = 0;   // one wave: the workspace bound is checked below
    const Plan p = make_plan(s);
    char* base = workspace(c->device);
    if (!base) fail(CCM_E_DEVICE, "no workspace on this device");

    // carve the plan's buffers out of the workspace (256-byte aligned)
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
      const uint64_t at = o;
      o = up256(o + std::max<uint64_t>(bytes, 1));
      return base + at;
    };
    PlanBuffers b;
    b.ingest = reinterpret_cast<IngestJob*>(take(p.ingest.size() * sizeof(IngestJob)));
    b.embed = reinterpret_cast<EmbedJob*>(take(p.embed.size() * sizeof(EmbedJob)));
    b.sample = reinterpret_cast<SampleJob*>(take(p.sample.size() * sizeof(SampleJob)));
    b.gather = reinterpret_cast<GatherJob*>(take(p.gather.size() * sizeof(GatherJob)));
    b.rz = reinterpret_cast<Realization*>(take(p.rz.size() * sizeof(Realization)));
    b.items = reinterpret_cast<Item*>(take(p.items.size() * sizeof(Item)));
    b.orders = reinterpret_cast<OrderJob*>(take(p.orders.size() * sizeof(OrderJob)));
    b.segoff = reinterpret_cast<int32_t*>(take(p.seg_off.size() * 4));
    b.s64 = reinterpret_cast<double*>(take(p.n64 * 8));
    b.s32 = reinterpret_cast<float*>(take(p.n32 * 4));
    b.iota = reinterpret_cast<int32_t*>(take(p.n_ord * 4));
    b.keys = reinterpret_cast<uint32_t*>(take(p.n_ord * 4));
    b.keys_out = reinterpret_cast<uint32_t*>(take(p.n_ord * 4));
    b.order = reinterpret_cast<int32_t*>(take(p.n_ord * 4));
    b.sort_temp = take(p.sort_temp);
    b.qord = reinterpret_cast<int32_t*>(take(p.n_qord * 4));
    b.start = reinterpret_cast<int32_t*>(take((uint64_t)p.n_slots * 4 * kWaves));
    b.emb = reinterpret_cast<float*>(take(p.n_emb * 4));
    b.lib = reinterpret_cast<int32_t*>(take(p.n_lib * 4));
    b.pts = reinterpret_cast<float*>(take(p.n_pts * 4));
    b.pj = reinterpret_cast<int32_t*>(take(p.n_pj * 4));
    b.partial = take((uint64_t)p.n_slots * sizeof(Moments));
    b.out = reinterpret_cast<double*>(take(p.n_out * 8));
    b.counter = reinterpret_cast<int*>(take(std::max<size_t>(64, p.launches.size()) * 4));
    if (o > kWorkspaceBytes)
      fail(CCM_E_NOMEM, "the call needs " + std::to_string(o) +
                            " bytes of workspace; the static workspace holds " +
                            std::to_string(kWorkspaceBytes));

    hipStream_t st = static_cast<hipStream_t>(stream);
    auto put = [&](void* dst, const void* src, size_t bytes) {
      if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    };
    put(b.ingest, p.ingest.data(), p.ingest.size() * sizeof(IngestJob));
    put(b.embed, p.embed.data(), p.embed.size() * sizeof(EmbedJob));
    put(b.sample, p.sample.data(), p.sample.size() * sizeof(SampleJob));
    put(b.gather, p.gather.data(), p.gather.size() * sizeof(GatherJob));
    put(b.rz, p.rz.data(), p.rz.size() * sizeof(Realization));
    put(b.items, p.items.data(), p.items.size() * sizeof(Item));
    put(b.orders, p.orders.data(), p.orders.size() * sizeof(OrderJob));
    put(b.segoff, p.seg_off.data(), p.seg_off.size() * 4);
    HIPCHK(hipMemcpyAsync(b.s64, X, N * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(b.s64 + N, Y, N * 8, hipMemcpyDeviceToDevice, st));
    enqueue_plan(c, p, b, {}, st, nullptr);
    const int64_t half = (int64_t)nL * r;
    HIPCHK(hipMemcpyAsync(rho_xy, b.out, half * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(rho_yx, b.out + half, half * 8, hipMemcpyDeviceToDevice, st));
    if (L_eff)
      for (int i = 0; i < nL; ++i) L_eff[i] = p.L_eff[i];
  });
}
