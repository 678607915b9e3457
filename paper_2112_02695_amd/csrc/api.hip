// C ABI entry points, context, workspace and table cache.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "collision_common.hpp"
#include "internal.hpp"

void* blr_ctx_t::arena_slice(const std::string& name, size_t bytes) {
  const size_t need = (std::max<size_t>(bytes, 256) + 255) / 256 * 256;
  auto it = arena_slices.find(name);
  if (it != arena_slices.end() && it->second.second >= need) return it->second.first;
  if (need > arena_cap - arena_used)
    throw blr::Error(BLR_ERR_ARG, "allocation-free call: workspace exceeds the static scratch (" +
                                      std::to_string(arena_cap) + " bytes)");
  void* p = arena_base + arena_used;
  arena_used += need;
  arena_slices[name] = {p, need};
  return p;
}

void* blr_ctx_t::buf(const std::string& name, size_t bytes) {
  if (arena_on) return arena_slice(name, bytes);
  if (bytes == 0) bytes = 256;
  auto& b = bufs[name];
  if (b.bytes < bytes) {
    if (capturing) {  // no allocation while a graph is recorded
      capture_broken = true;
      return b.p;
    }
    ++buf_gen;
    if (b.p) {
      BLR_HIP(hipStreamSynchronize(stream));
      BLR_HIP(hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
    }
    BLR_HIP(hipMalloc(&b.p, bytes));
    b.bytes = bytes;
  }
  return b.p;
}

void* blr_ctx_t::upload(const std::string& name, const void* host, size_t bytes) {
  // one device copy per distinct content (FNV-1a of the bytes in the name):
  // work recorded into a graph keeps reading its own index arrays
  const unsigned char* hb = (const unsigned char*)host;
  uint64_t hsh = 1469598103934665603ull;
  for (size_t k = 0; k < bytes; ++k) hsh = (hsh ^ hb[k]) * 1099511628211ull;
  const std::string key = name + "#" + std::to_string(bytes) + "#" + std::to_string(hsh);
  void* dst = buf(key, bytes);
  if (bytes == 0) return dst;
  if (arena_on) {
    // from pageable host memory: the copy has read the source when it returns
    BLR_HIP(hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, stream));
    return dst;
  }
  auto& last = uploaded[key];
  if (last.first == dst && last.second.size() == bytes && std::memcmp(last.second.data(), hb, bytes) == 0)
    return dst;
  if (capturing) {  // a staged copy cannot be replayed
    capture_broken = true;
    return dst;
  }
  StageSlot& sl = stage[stage_next];
  stage_next = (stage_next + 1) % kStageSlots;
  if (sl.done) BLR_HIP(hipEventSynchronize(sl.done));
  if (sl.bytes < bytes) {
    if (sl.p) BLR_HIP(hipHostFree(sl.p));
    sl.p = nullptr;
    sl.bytes = 0;
    const size_t want = std::max<size_t>(bytes, 64 << 10);
    BLR_HIP(hipHostMalloc(&sl.p, want));
    sl.bytes = want;
  }
  std::memcpy(sl.p, host, bytes);
  BLR_HIP(hipMemcpyAsync(dst, sl.p, bytes, hipMemcpyHostToDevice, stream));
  if (!sl.done) BLR_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  BLR_HIP(hipEventRecord(sl.done, stream));
  last.first = dst;
  last.second.assign(hb, hb + bytes);
  return dst;
}

int blr_ctx_t::cu_count() {
  if (ncu <= 0) {
    BLR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    if (ncu <= 0) ncu = 1;
  }
  return ncu;
}

void* blr_ctx_t::host_readback(size_t bytes) {
  if (readback_bytes < bytes) {
    if (capturing) {
      capture_broken = true;
      return readback;
    }
    ++buf_gen;
    if (readback) {
      BLR_HIP(hipStreamSynchronize(stream));
      BLR_HIP(hipHostFree(readback));
    }
    readback = nullptr;
    readback_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 4096);
    BLR_HIP(hipHostMalloc(&readback, want));
    readback_bytes = want;
  }
  return readback;
}

void blr_ctx_t::release_all() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs.clear();
  tables.clear();
  for (auto& sl : stage) {
    if (sl.p) (void)hipHostFree(sl.p);
    if (sl.done) (void)hipEventDestroy(sl.done);
    sl = StageSlot{};
  }
  uploaded.clear();
  if (readback) (void)hipHostFree(readback);
  readback = nullptr;
  readback_bytes = 0;
  for (auto& g : graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.exec2) (void)hipGraphExecDestroy(g.exec2);
  }
  graphs.clear();
  if (cap_stream) {
    (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  timer.release();
}

namespace blr {

hipEvent_t KernelTimer::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  BLR_HIP(hipEventCreate(&e));
  return e;
}
void KernelTimer::begin(hipStream_t s, const std::string& name, double bytes) {
  if (!on) return;
  Rec r{name, take(), take(), bytes};
  BLR_HIP(hipEventRecord(r.a, s));
  pending.push_back(r);
}
void KernelTimer::end(hipStream_t s) {
  if (!on || pending.empty()) return;
  BLR_HIP(hipEventRecord(pending.back().b, s));
}
void KernelTimer::collect() {
  for (auto& r : pending) {
    BLR_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    BLR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto it = acc.find(r.name);
    if (it == acc.end()) {
      order.push_back(r.name);
      acc[r.name] = Acc{};
      it = acc.find(r.name);
    }
    it->second.ms += ms;
    it->second.bytes += r.bytes;
    it->second.launches += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}
void KernelTimer::release() {
  for (auto& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pending.clear();
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

DevTables::~DevTables() {
  for (void* p : owned)
    if (p) (void)hipFree(p);
}

// Copies on the context's own stream (never the legacy default stream, which
// another host thread's graph recording would forbid), then waits for it.
template <typename T>
static void* upload_vec(DevTables& t, const std::vector<T>& v, hipStream_t s) {
  void* p = nullptr;
  BLR_HIP(hipMalloc(&p, std::max<size_t>(v.size() * sizeof(T), 16)));
  t.owned.push_back(p);
  if (!v.empty()) {
    BLR_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    BLR_HIP(hipStreamSynchronize(s));
  }
  return p;
}

template <typename T>
static std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// Allocation-free mode: the host tables are built once per configuration and
// copied into the context's arena at every call (the arena is shared by all
// calls on the device, so nothing left there by an earlier call is trusted).
const HostTables& arena_host_tables(blr_ctx ctx, const blr_vgrid& vg, int prec) {
  auto& t = ctx->arena_tables;
  const blr_vgrid& o = t ? t->vg : vg;
  const bool same = t && t->prec == prec && o.d == vg.d && o.n == vg.n && o.L == vg.L &&
                    o.R == vg.R && o.C == vg.C && o.gamma == vg.gamma && o.m_rho == vg.m_rho &&
                    o.m_sigma == vg.m_sigma && o.aniso_n == vg.aniso_n &&
                    std::memcmp(o.aniso, vg.aniso, sizeof(double) * 5) == 0 &&
                    (o.flags & BLR_CARLEMAN) == (vg.flags & BLR_CARLEMAN);
  if (!same) {
    t = std::make_unique<DevTables>();
    t->h = build_tables(vg);
    t->prec = prec;
    t->vg = vg;
  }
  return t->h;
}

static const DevTables& arena_tables(blr_ctx ctx, const blr_vgrid& vg, int prec) {
  const HostTables& h = arena_host_tables(ctx, vg, prec);
  DevTables* t = ctx->arena_tables.get();
  auto put = [&](const char* nm, const void* data, size_t bytes) -> void* {
    void* p = ctx->arena_slice(std::string("tab.") + nm, bytes);
    if (bytes) BLR_HIP(hipMemcpyAsync(p, data, bytes, hipMemcpyHostToDevice, ctx->stream));
    return p;
  };
  auto putv = [&](const char* nm, const std::vector<double>& v) -> void* {
    if (prec == BLR_FP32) {
      const std::vector<float> f(v.begin(), v.end());
      return put(nm, f.data(), f.size() * sizeof(float));
    }
    return put(nm, v.data(), v.size() * sizeof(double));
  };
  std::vector<double> wbp(h.nbp);
  for (int p = 0; p < h.nbp; ++p) wbp[p] = h.wsig[h.bp_b[p]];
  t->phase = putv("phase", h.phase);
  t->fw = putv("fw", h.fw);
  t->gloss = putv("gloss", h.gloss);
  t->wbp = putv("wbp", wbp);
  t->filt = h.carleman ? putv("filt", h.filt) : nullptr;
  t->atab = h.aniso_n > 0 ? putv("atab", h.atab) : nullptr;
  t->bp_b = (int*)put("bp_b", h.bp_b.data(), h.bp_b.size() * sizeof(int));
  t->bp_bb = (int*)put("bp_bb", h.bp_bb.data(), h.bp_bb.size() * sizeof(int));
  return *t;
}

const DevTables& get_tables(blr_ctx ctx, const blr_vgrid& vg, int prec) {
  validate_vgrid(vg);
  if (ctx->arena_on) return arena_tables(ctx, vg, prec);
  const int ms = vg.m_sigma ? vg.m_sigma : (vg.d == 2 ? 8 : 38);
  const int form = (vg.flags & BLR_CARLEMAN) ? 1 : 0;
  // every field the tables depend on, doubles by their bit patterns
  std::string key;
  auto put = [&key](const void* p, size_t b) { key.append((const char*)p, b); };
  const int ints[6] = {vg.d, vg.n, vg.m_rho, ms, prec, form};
  const double dbl[4] = {vg.L, vg.R, vg.C, vg.gamma};
  put(ints, sizeof(ints));
  put(dbl, sizeof(dbl));
  put(&vg.aniso_n, sizeof(vg.aniso_n));
  put(vg.aniso, sizeof(double) * (vg.aniso_n > 0 ? vg.aniso_n : 0));
  auto it = ctx->tables.find(key);
  if (it != ctx->tables.end()) return *it->second;
  auto t = std::make_unique<DevTables>();
  t->h = build_tables(vg);
  t->prec = prec;
  const HostTables& h = t->h;
  std::vector<double> wbp(h.nbp);
  for (int p = 0; p < h.nbp; ++p) wbp[p] = h.wsig[h.bp_b[p]];
  if (prec == BLR_FP32) {
    t->phase = upload_vec(*t, cast_vec<float>(h.phase), ctx->stream);
    t->fw = upload_vec(*t, cast_vec<float>(h.fw), ctx->stream);
    t->gloss = upload_vec(*t, cast_vec<float>(h.gloss), ctx->stream);
    t->wbp = upload_vec(*t, cast_vec<float>(wbp), ctx->stream);
  } else {
    t->phase = upload_vec(*t, h.phase, ctx->stream);
    t->fw = upload_vec(*t, h.fw, ctx->stream);
    t->gloss = upload_vec(*t, h.gloss, ctx->stream);
    t->wbp = upload_vec(*t, wbp, ctx->stream);
  }
  if (h.carleman) {
    if (prec == BLR_FP32) t->filt = upload_vec(*t, cast_vec<float>(h.filt), ctx->stream);
    else t->filt = upload_vec(*t, h.filt, ctx->stream);
  }
  if (h.aniso_n > 0) {
    if (prec == BLR_FP32) t->atab = upload_vec(*t, cast_vec<float>(h.atab), ctx->stream);
    else t->atab = upload_vec(*t, h.atab, ctx->stream);
  }
  t->bp_b = (int*)upload_vec(*t, h.bp_b, ctx->stream);
  t->bp_bb = (int*)upload_vec(*t, h.bp_bb, ctx->stream);
  auto& slot = ctx->tables[key];
  slot = std::move(t);
  return *slot;
}

}  // namespace blr

// ------------------------------------------------- allocation-free calls --
// The device region of blr_collision_pairs_noalloc: one array per device, part
// of the library's code object (so it exists, on each device the library runs
// on, from the library's first use there until the process ends).  Host code
// never passes `scratch` itself (its host-side name is not a device address):
// blr_create resolves the array's device address once per device, with that
// device current, and calls use that address.
static constexpr size_t kScratchBytes = (size_t)BLR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, std::pair<hipError_t, void*>> g_scratch_addr;  // device -> (status, address)

// Resolves the scratch array's address on `device` (current) once.
void resolve_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr.count(device)) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  g_scratch_addr[device] = {e, e == hipSuccess ? ptr : nullptr};
}

void* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  blr::require(it != g_scratch_addr.end(), "scratch address not resolved for this device",
               BLR_ERR_HIP);
  if (it->second.first != hipSuccess)
    throw blr::Error(BLR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(it->second.first));
  return it->second.second;
}

// Arena mode for the duration of one call (left on every exit path).
struct ArenaScope {
  blr_ctx c;
  ArenaScope(blr_ctx ctx, void* base, size_t cap) : c(ctx) {
    c->arena_on = true;
    c->arena_base = (char*)base;
    c->arena_cap = cap;
    c->arena_used = 0;
    c->arena_slices.clear();
  }
  ~ArenaScope() {
    c->arena_on = false;
    c->arena_slices.clear();
  }
};
}  // namespace

// ----------------------------------------------------------------- C ABI --
template <class F>
static blr_status guarded(blr_ctx ctx, F&& f) {
  if (!ctx) return BLR_ERR_ARG;
  ctx->err.clear();
  try {
    BLR_HIP(hipSetDevice(ctx->device));
    f();
    return BLR_OK;
  } catch (const blr::Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return BLR_ERR_NOMEM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return BLR_ERR_HIP;
  }
}

extern "C" {

blr_status blr_create(int device, void* hip_stream, blr_ctx* out) {
  if (!out) return BLR_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BLR_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return BLR_ERR_HIP;
  blr_ctx c = new (std::nothrow) blr_ctx_t();
  if (!c) return BLR_ERR_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  resolve_scratch(device);
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return BLR_ERR_HIP;
    }
  *out = c;
  return BLR_OK;
}

blr_status blr_destroy(blr_ctx ctx) {
  if (!ctx) return BLR_ERR_ARG;
  (void)hipSetDevice(ctx->device);
  ctx->release_all();
  delete ctx;
  return BLR_OK;
}

const char* blr_last_error(blr_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

blr_status blr_workspace_bytes(blr_ctx ctx, const blr_vgrid* vg, int32_t r_max,
                               blr_precision prec, size_t* out) {
  return guarded(ctx, [&] {
    blr::require(vg && out, "null pointer argument");
    blr::require(r_max >= 1 && r_max <= 64, "r_max must be in [1, 64]");
    blr::require(prec == BLR_FP32 || prec == BLR_FP64, "bad precision");
    *out = blr::collision_workspace_bytes(*vg, r_max, prec);
  });
}

blr_status blr_collision_pairs(blr_ctx ctx, const blr_vgrid* vg, blr_precision prec,
                               const void* V, int32_t r, const int32_t* pairs,
                               int32_t npairs, void* Q_out) {
  return guarded(ctx, [&] {
    blr::require(vg != nullptr, "null vgrid");
    blr::require(prec == BLR_FP32 || prec == BLR_FP64, "bad precision");
    blr::collision_pairs(ctx, *vg, prec, V, r, pairs, npairs, Q_out);
  });
}

blr_status blr_collision_pairs_noalloc(blr_ctx ctx, const blr_vgrid* vg, blr_precision prec,
                                       const void* V, int32_t r, const int32_t* pairs,
                                       int32_t npairs, void* Q_out) {
  return guarded(ctx, [&] {
    blr::require(vg != nullptr, "null vgrid");
    blr::require(prec == BLR_FP32 || prec == BLR_FP64, "bad precision");
    blr::require(r >= 1 && r <= 64, "r must be in [1, 64]");
    blr::require(npairs >= 0 && npairs <= 4096, "npairs must be in [0, 4096]");
    blr::require(npairs == 0 || (pairs && V && Q_out), "null pointer argument");
    if (npairs == 0) return;
    blr::validate_vgrid(*vg);
    blr::require(!(vg->flags & BLR_DEALIAS), "allocation-free call: BLR_DEALIAS is not available",
                 BLR_ERR_UNSUPPORTED);
    void* base = scratch_address(ctx->device);
    // the whole call's workspace must fit before anything is issued
    const blr::HostTables& h = blr::arena_host_tables(ctx, *vg, prec);
    const size_t need = blr::collision_call_bytes(h, prec, r, pairs, npairs, vg->flags);
    blr::require(need <= kScratchBytes,
                 "allocation-free call needs " + std::to_string(need) +
                     " bytes of workspace; the static scratch holds " +
                     std::to_string(kScratchBytes));
    ArenaScope scope(ctx, base, kScratchBytes);
    blr::collision_pairs(ctx, *vg, prec, V, r, pairs, npairs, Q_out);
  });
}

blr_status blr_timing(blr_ctx ctx, int32_t mode) {
  return guarded(ctx, [&] {
    blr::require(mode >= 0 && mode <= 2, "mode must be 0 (off), 1 (on) or 2 (reset)");
    if (mode == 2) {
      ctx->timer.collect();
      ctx->timer.acc.clear();
      ctx->timer.order.clear();
      return;
    }
    ctx->timer.on = mode == 1;
  });
}

blr_status blr_timing_read(blr_ctx ctx, int32_t idx, char* name, int32_t name_len, double* ms,
                           int64_t* launches, double* bytes) {
  return guarded(ctx, [&] {
    blr::require(name && name_len > 0 && ms && launches && bytes, "null pointer argument");
    ctx->timer.collect();
    blr::require(idx >= 0 && idx < (int)ctx->timer.order.size(), "timer index out of range");
    const std::string& nm = ctx->timer.order[idx];
    const auto& v = ctx->timer.acc[nm];
    std::snprintf(name, name_len, "%s", nm.c_str());
    *ms = v.ms;
    *launches = v.launches;
    *bytes = v.bytes;
  });
}

}  // extern "C"
