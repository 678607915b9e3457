// Internal declarations of the blr library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/blr.h"

namespace blr {

// Error carrying a blr_status across the C++ layers; caught at the C ABI.
struct Error : std::runtime_error {
  blr_status code;
  Error(blr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define BLR_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      if (e_ == hipErrorOutOfMemory)                                                    \
        throw ::blr::Error(BLR_ERR_NOMEM, std::string(#call) + ": out of device memory"); \
      throw ::blr::Error(BLR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                                   \
  } while (0)

#define BLR_CHECK_LAUNCH() BLR_HIP(hipGetLastError())

inline void require(bool ok, const std::string& msg, blr_status code = BLR_ERR_ARG) {
  if (!ok) throw Error(code, msg);
}

// ----------------------------------------------------------------- tables --
// Host-side (FP64) description of one velocity discretisation.
struct HostTables {
  int d = 0, N = 0, n = 0, mrho = 0, msig = 0, nbp = 0, nkk = 0;
  double L = 0, R = 0, C = 0, gamma = 0, dv = 0;
  std::vector<double> rho, wrho, cw;          // radial nodes, weights, w*rho^(d-1)
  std::vector<double> sig, wsig;              // msig x 3, msig
  std::vector<int> bp_b, bp_bb;               // antipodal pairs (b, bbar), b < bbar
  std::vector<double> phase;                  // (mrho*nbp) x d x N x 2 : exp(-i th sigma_b,ax k)
  std::vector<double> fw;                     // mrho x nkk : cw B A_d(th |k|) / n
  std::vector<double> gloss;                  // n     : G-(k) (DFT order)
  std::vector<double> minv;                   // (d+2)^2 : (C C^T)^-1, C rows dv^d{1,v,|v|^2}
  // Carleman form (BLR_CARLEMAN): one "radial node", nbp direction pairs of
  // filtered fields, filt = nbp x n complex multipliers (DFT order) whose
  // inverse transform W gives the pair's two fields as Re W - Im W and
  // Re W + Im W; gloss holds beta(l, l); phase and fw are unused.
  bool carleman = false;
  std::vector<double> filt;                   // nbp x n x 2
  // anisotropic kernel (aniso_n > 0): per radial node a and antipodal pair p
  // the spectral weight cw_a (F_ab + F_abbar)(k) / (2 n) of the pair's product
  // (real: only even angular components survive the symmetrisation); gloss
  // carries aniso[0]; fw is unused.
  int aniso_n = 0;
  double aniso[5] = {0, 0, 0, 0, 0};
  std::vector<double> atab;                   // mrho x nbp x n
};

HostTables build_tables(const blr_vgrid& vg);
double bessel_j0(double z);
void gauss_legendre(int m, double R, std::vector<double>& x, std::vector<double>& w);

// Device copies of the tables in one precision.
struct DevTables {
  HostTables h;
  int prec = 0;
  void* phase = nullptr;   // T2 : (mrho*nbp) x d x N
  void* fw = nullptr;      // T  : mrho x nkk
  void* gloss = nullptr;   // T  : n
  void* wbp = nullptr;     // T  : nbp sphere weights of the antipodal pairs
  int* bp_b = nullptr;     // nbp
  int* bp_bb = nullptr;    // nbp
  void* filt = nullptr;    // T2 : nbp x n (Carleman form only)
  void* atab = nullptr;    // T  : mrho x nbp x n (anisotropic kernel only)
  blr_vgrid vg{};          // the grid these tables describe (allocation-free mode)
  std::vector<void*> owned;
  ~DevTables();
};

// ---------------------------------------------------------------- context --
struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

// Optional per-kernel timing: launches bracketed by HIP events on the
// context stream, accumulated per kernel name when read.
struct KernelTimer {
  bool on = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> order;
  struct Acc {
    double ms = 0, bytes = 0;
    long launches = 0;
  };
  std::map<std::string, Acc> acc;
  hipEvent_t take();
  void begin(hipStream_t s, const std::string& name, double bytes);
  void end(hipStream_t s);
  void collect();
  void release();
};

}  // namespace blr

struct blr_ctx_t {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, std::unique_ptr<blr::DevTables>> tables;  // by grid, kernel and precision
  std::map<std::string, blr::Buffer> bufs;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t calls = 0;

  // pinned staging for small per-call host->device uploads: a ring of slots,
  // each reused only after its previous copy has completed
  struct StageSlot {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
  };
  static constexpr int kStageSlots = 8;
  StageSlot stage[kStageSlots];
  int stage_next = 0;
  // last content uploaded to each named buffer (identical uploads are skipped)
  std::map<std::string, std::pair<void*, std::vector<unsigned char>>> uploaded;
  // pinned host buffer for small device->host read-backs
  void* readback = nullptr;
  size_t readback_bytes = 0;
  // number of boundary basis functions added by the previous adaptive step
  int add_hint = -1;
  // FP64 defect of the FP32 pair collisions kept by the last refresh step
  // (BLR_STEP_FP64_DEFECT): the basis rank at its collisions (0: none kept)
  // and its velocity grid; the defect and the basis live in the buffers
  // "dlr.defect.D" and "dlr.defect.V"
  int defect_r = 0;
  blr_vgrid defect_vg{};
  // the 2D step's boundary-factor SVD: the size of the right singular vectors
  // kept in "dlr.d2.Wwarm" (0: none) and the steps since a fresh start
  int bsvd_n = 0, bsvd_age = 0;
  // compute units of the device (queried once)
  int ncu = 0;
  int cu_count();
  // bumped whenever a workspace buffer or the read-back buffer moves: graphs
  // recorded before hold stale addresses
  uint64_t buf_gen = 0;
  // step graphs: the device work of one step attempt recorded once per
  // configuration (key) and replayed; capture runs on cap_stream
  struct StepGraph {
    std::string key;
    uint64_t gen = 0;
    int seen = 0;
    hipGraphExec_t exec = nullptr;
    // where the recorded work leaves its results
    int r = 0, nrb = 0;
    double *X1 = nullptr, *V1 = nullptr, *Snew = nullptr, *U = nullptr, *Wm = nullptr,
           *sgd = nullptr, *hb = nullptr;
    // a step whose collisions go through collide_hook is two graphs: exec up
    // to the collisions, exec2 after them; the collisions' arguments
    hipGraphExec_t exec2 = nullptr;
    blr_vgrid cvg{};
    const float* cV = nullptr;
    int cr = 0;
    std::vector<int32_t> cpairs;
    float* cQ = nullptr;
  };
  std::vector<StepGraph> graphs;
  hipStream_t cap_stream = nullptr;
  bool capturing = false;
  bool capture_broken = false;  // an operation that cannot be recorded was requested
  blr::KernelTimer timer;

  // Allocation-free mode (blr_collision_pairs_noalloc): while arena_on, buf()
  // and upload() hand out named 256-byte-aligned slices of the device region
  // [arena_base, arena_base + arena_cap) instead of allocating, and
  // get_tables() copies the tables into it (arena_tables).  A name asked for
  // twice in one call gets the same slice.
  bool arena_on = false;
  char* arena_base = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  std::map<std::string, std::pair<void*, size_t>> arena_slices;
  std::unique_ptr<blr::DevTables> arena_tables;
  void* arena_slice(const std::string& name, size_t bytes);

  // Served batches (blr_server with batch_collisions): the fused FP32 path
  // fixes its radial-node grouping of the pair transforms (so a pair's result
  // does not depend on how many pairs share the launch) and picks the
  // sigma-sum tile width by timing the candidates once per shape.
  bool batch_mode = false;
  std::map<std::string, int> tuned_tile;
  // When set, the FP32 collisions of a step go through this hook (a served
  // solve's collisions batched with those of the other live solves).
  struct CollideHook {
    virtual void collide(blr_ctx ctx, const blr_vgrid& vg, const float* V, int r,
                         const std::vector<int32_t>& pairs, float* Q) = 0;
    virtual ~CollideHook() = default;
  };
  CollideHook* collide_hook = nullptr;
  // while a step with collide_hook is recorded: the graph up to its
  // collisions (the recording then continues after them) and their arguments
  hipGraph_t split_g1 = nullptr;
  blr_vgrid split_vg{};
  const float* split_V = nullptr;
  int split_r = 0;
  std::vector<int32_t> split_pairs;
  float* split_Q = nullptr;

  void* buf(const std::string& name, size_t bytes);  // grow-only named workspace
  // copy a small host array to a named device buffer, asynchronously
  void* upload(const std::string& name, const void* host, size_t bytes);
  // pinned host memory of at least `bytes` for read-backs (grow-only)
  void* host_readback(size_t bytes);
  void release_all();
};

namespace blr {

const DevTables& get_tables(blr_ctx ctx, const blr_vgrid& vg, int prec);
// host tables of the allocation-free mode (cached in the context)
const HostTables& arena_host_tables(blr_ctx ctx, const blr_vgrid& vg, int prec);
void validate_vgrid(const blr_vgrid& vg);

// collision pipeline (collision.hip)
void collision_pairs(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int r,
                     const int32_t* pairs_dev, int npairs, void* Q);
size_t collision_workspace_bytes(const blr_vgrid& vg, int r, int prec);
// The FP32 pair collisions of several bases on one velocity grid in shared
// launches: the bases are laid side by side (at most 64 functions and 4096
// pairs per launch sequence) and each job's rows copied back to its Q.
struct BatchJob {
  const float* V;
  int r;
  std::vector<int32_t> pairs;  // 2 P indices into the job's own basis
  float* Q;                    // P rows of n
};
void collision_batch(blr_ctx ctx, const blr_vgrid& vg, const std::vector<BatchJob>& jobs);
// the fused FP32 path takes this grid (3D, n in {16, 24, 32}, 38 directions,
// the (rho, sigma) form with an isotropic kernel, no de-aliasing)
bool fused_f32_grid(const blr_vgrid& vg);
// Q_s(V_i, V_i) for the rows i = 0..rows-1 of V into the rows of Q (the
// full-tensor step's cells): the pipeline of collision_pairs without its
// 64-row limit, since a pair list of rows (i, i) needs no pair tiles.
constexpr int kMaxSelfRows = 1024;
void collision_self(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int rows, void* Q);
// Upper bound of the device bytes collision_pairs takes from buf()/upload()
// and the tables for this call (each slice rounded up to 256 bytes).
size_t collision_call_bytes(const HostTables& h, int prec, int r, const int32_t* pairs, int npairs,
                            uint32_t flags);
// Bytes of the device tables of one precision (rounded as above).
size_t table_bytes(const HostTables& h, int prec);

// DLR step and steady solve (dlr.hip)
void dlr_step(blr_ctx ctx, const blr_problem* pb, blr_state* st, const blr_step_params* sp,
              blr_step_info* info);
void steady_solve(blr_ctx ctx, const blr_problem* pb, blr_state* state, const blr_solve_params* p,
                  blr_solve_info* info, const std::atomic<bool>* cancel = nullptr);
size_t solve_workspace_bytes(const blr_vgrid& vg, int nx, int r_cap, bool fp64_collision,
                             bool defect = false);

}  // namespace blr
