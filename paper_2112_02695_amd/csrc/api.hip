// C ABI entry points, context, workspace and table cache.
#include <cmath>
#include <cstring>

#include "collision_common.hpp"
#include "internal.hpp"

void* blr_ctx_t::buf(const std::string& name, size_t bytes) {
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
  for (auto& g : graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
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

const DevTables& get_tables(blr_ctx ctx, const blr_vgrid& vg, int prec) {
  validate_vgrid(vg);
  const int ms = vg.m_sigma ? vg.m_sigma : (vg.d == 2 ? 8 : 38);
  const int form = (vg.flags & BLR_CARLEMAN) ? 1 : 0;
  auto key = std::make_tuple(vg.d, vg.n, vg.L, vg.R, vg.C, vg.gamma, vg.m_rho, ms, prec, form);
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
  t->bp_b = (int*)upload_vec(*t, h.bp_b, ctx->stream);
  t->bp_bb = (int*)upload_vec(*t, h.bp_bb, ctx->stream);
  auto& slot = ctx->tables[key];
  slot = std::move(t);
  return *slot;
}

}  // namespace blr

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
