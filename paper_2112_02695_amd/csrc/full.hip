// Full-tensor reference step on the GPU: the discretisation the low-rank
// method is projected from (first-order upwind in x, eq. scheme:fullupwind of
// Sec. 2.2, forward Euler in time, walls of Sec. 2.3), with the collision
// term Q(f(x_p,.), f(x_p,.)) of every cell evaluated by the pair pipeline
// (the cells of a chunk are its basis, the pairs are (p, p)).  err_full is
// eq. err full grid.
//
// F is row-major nx x n^d FP64 (row p = cell p); the update is written to a
// second array and copied back once every cell's collision term is in, since
// the transport of cell p reads cells p - 1 and p + 1.
#include <cmath>
#include <vector>

#include "collision_common.hpp"
#include "obstacle.hpp"
#include "walls.hpp"

namespace blr {
namespace fk {

constexpr int kChunk = 64;  // cells per collision call (the pair pipeline's basis limit)

// Boundary-function scale of each side: rho_w of a diffusive wall from the
// cell next to it (Sec. 2.3), 1 for an inflow boundary.  One block per side.
__global__ __launch_bounds__(1024) void k_full_wall_rho(const double* __restrict__ F, int nx, int n,
                                                        const double* __restrict__ fL,
                                                        const double* __restrict__ fR, int wl,
                                                        int wr, double L, double dv, int plane,
                                                        double* __restrict__ rho) {
  const int side = blockIdx.x;
  if (!(side == 0 ? wl : wr)) {
    if (threadIdx.x == 0) rho[side] = 1.0;
    return;
  }
  __shared__ double red[1024 / 64 + 1];
  const double v = wall::density<1024>(side, F + (long)(side ? nx - 1 : 0) * n, side ? fR : fL, n,
                                       L, dv, plane, red);
  if (threadIdx.x == 0) rho[side] = v;
}

// F_new = F - dt (v1+ (F_p - F_{p-1}) + v1- (F_{p+1} - F_p)) / dx + dt Q_p for the
// cells p0 .. p0 + gridDim.y - 1; the ghost F_{-1} is rho[0] f_L where v1 > 0
// and F_{nx} is rho[1] f_R where v1 < 0 (the outflow halves multiply a zero
// velocity part).  Writes each block's sum of (F_new - F)^2 (wave sums, then
// the waves in order) to part[p * gridDim.x + blockIdx.x].
template <typename TQ>
__global__ __launch_bounds__(256) void k_full_update(const double* __restrict__ F, int nx, int n,
                                                     int p0, const TQ* __restrict__ Q,
                                                     const double* __restrict__ fL,
                                                     const double* __restrict__ fR,
                                                     const double* __restrict__ rho, double dt,
                                                     double dx, double L, double dv, int plane,
                                                     double* __restrict__ Fn,
                                                     double* __restrict__ part) {
  __shared__ double ws[4];
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int p = p0 + blockIdx.y;
  double e2 = 0.0;
  if (q < n) {
    const double v1 = -L + (q / plane) * dv;
    const double* fp = F + (long)p * n + q;
    const double f = fp[0];
    const double fm = p > 0 ? fp[-n] : (v1 > 0 ? rho[0] * fL[q] : f);
    const double fn = p < nx - 1 ? fp[n] : (v1 < 0 ? rho[1] * fR[q] : f);
    const double vp = v1 > 0 ? v1 : 0.0, vm = v1 < 0 ? v1 : 0.0;
    const double d = -dt * (vp * (f - fm) + vm * (fn - f)) / dx +
                     dt * (double)Q[(long)blockIdx.y * n + q];
    Fn[(long)p * n + q] = f + d;
    e2 = d * d;
  }
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_down(e2, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[(long)p * gridDim.x + blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// ------------------------------------------------------------ 2D space
// Boundary functions of the four faces (x_lo, x_hi, y_lo, y_hi); bit k of
// `rows`: face k holds one row per face cell.
struct Faces {
  const double* f[4];
  int rows;
  __device__ __forceinline__ const double* row(int k, int c, int n) const {
    return f[k] + (((rows >> k) & 1) ? (long)c * n : 0L);
  }
};

// rho of every face cell (x_lo: ny cells, x_hi: ny, y_lo: nx, y_hi: nx, in
// that order, then the obstacle's faces): rho_w of a diffusive wall from the
// adjacent gas cell's distribution (Sec. 2.3), 1 on an inflow face.  One
// block per face.
__global__ __launch_bounds__(1024) void k_full_face_rho2d(const double* __restrict__ F, int nx,
                                                          int ny, int n, Faces fc, int walls,
                                                          Obs2 ob, double L, double dv, int plane,
                                                          int stride1, int N,
                                                          double* __restrict__ rho) {
  const int b = blockIdx.x;
  __shared__ double red[1024 / 64 + 1];
  if (b >= ob.nface) {
    const int i = b - ob.nface;
    const long cell = ob.face[2 * i];
    const int k = ob.face[2 * i + 1];
    const double v = wall::density_face<1024>((k % 2 == 0) ? -1.0 : 1.0, F + cell * n, ob.f, n, L,
                                              dv, k < 2 ? plane : stride1, N, red);
    if (threadIdx.x == 0) rho[b] = v;
    return;
  }
  int k, c;
  if (b < ny) {
    k = 0; c = b;
  } else if (b < 2 * ny) {
    k = 1; c = b - ny;
  } else if (b < 2 * ny + nx) {
    k = 2; c = b - 2 * ny;
  } else {
    k = 3; c = b - 2 * ny - nx;
  }
  if (!((walls >> k) & 1)) {
    if (threadIdx.x == 0) rho[b] = 1.0;
    return;
  }
  const long cell = k == 0 ? c : k == 1 ? (long)(nx - 1) * ny + c : k == 2 ? (long)c * ny
                                                                         : (long)c * ny + ny - 1;
  if (ob.is_solid(cell)) {    // no gas next to this face cell
    if (threadIdx.x == 0) rho[b] = 0.0;
    return;
  }
  const double v = wall::density_face<1024>((k % 2 == 0) ? -1.0 : 1.0, F + cell * n,
                                            fc.row(k, c, n), n, L, dv, k < 2 ? plane : stride1,
                                            N, red);
  if (threadIdx.x == 0) rho[b] = v;
}

// The update of k_full_update on the rectangle: cells p0 .. p0 + gridDim.y - 1
// (p = ix ny + iy), upwind differences along x (v_1) and y (v_2), ghosts
// rho f_face on the incoming half of a face (the cell itself elsewhere: that
// half multiplies a zero velocity part), also where the neighbour is solid
// (rho of that obstacle face times the obstacle's Maxwellian).  Solid cells
// hold no gas: F_new = 0 there.
template <typename TQ>
__global__ __launch_bounds__(256) void k_full_update2d(const double* __restrict__ F, int nx,
                                                       int ny, int n, long p0,
                                                       const TQ* __restrict__ Q, Faces fc, Obs2 ob,
                                                       const double* __restrict__ rho, double dt,
                                                       double dx, double dy, double L, double dv,
                                                       int plane, int stride1, int N,
                                                       double* __restrict__ Fn,
                                                       double* __restrict__ part) {
  __shared__ double ws[4];
  const int q = blockIdx.x * 256 + threadIdx.x;
  const long p = p0 + blockIdx.y;
  const int ix = (int)(p / ny), iy = (int)(p % ny);
  double e2 = 0.0;
  if (q < n) {
    const double v1 = -L + (q / plane) * dv;
    const double v2 = -L + ((q / stride1) % N) * dv;
    const double* fp = F + p * n + q;
    const double f = fp[0];
    const long sx = (long)ny * n;
    const int bxm = ob.towards(p, 0), bxp = ob.towards(p, 1);
    const int bym = ob.towards(p, 2), byp = ob.towards(p, 3);
    const double fxm = ix > 0 ? (bxm >= 0 ? (v1 > 0 ? rho[bxm] * ob.f[q] : f) : fp[-sx])
                              : (v1 > 0 ? rho[iy] * fc.row(0, iy, n)[q] : f);
    const double fxp = ix < nx - 1 ? (bxp >= 0 ? (v1 < 0 ? rho[bxp] * ob.f[q] : f) : fp[sx])
                                   : (v1 < 0 ? rho[ny + iy] * fc.row(1, iy, n)[q] : f);
    const double fym = iy > 0 ? (bym >= 0 ? (v2 > 0 ? rho[bym] * ob.f[q] : f) : fp[-n])
                              : (v2 > 0 ? rho[2 * ny + ix] * fc.row(2, ix, n)[q] : f);
    const double fyp = iy < ny - 1 ? (byp >= 0 ? (v2 < 0 ? rho[byp] * ob.f[q] : f) : fp[n])
                                   : (v2 < 0 ? rho[2 * ny + nx + ix] * fc.row(3, ix, n)[q] : f);
    const double v1p = v1 > 0 ? v1 : 0.0, v1m = v1 < 0 ? v1 : 0.0;
    const double v2p = v2 > 0 ? v2 : 0.0, v2m = v2 < 0 ? v2 : 0.0;
    const double d = ob.is_solid(p) ? -f
                                    : -dt * ((v1p * (f - fxm) + v1m * (fxp - f)) / dx +
                                             (v2p * (f - fym) + v2m * (fyp - f)) / dy) +
                                          dt * (double)Q[(long)blockIdx.y * n + q];
    Fn[p * n + q] = f + d;
    e2 = d * d;
  }
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_down(e2, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[p * gridDim.x + blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// err = sqrt(w sum part) over cnt partials, one block, fixed order
__global__ __launch_bounds__(256) void k_err_total(const double* __restrict__ part, long cnt,
                                                   double w, double* __restrict__ err) {
  __shared__ double ws[4];
  double s = 0.0;
  for (long i = threadIdx.x; i < cnt; i += 256) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) err[0] = std::sqrt(w * (((ws[0] + ws[1]) + ws[2]) + ws[3]));
}

__global__ void k_cast_f32(const double* __restrict__ in, long count, float* __restrict__ out) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < count) out[e] = (float)in[e];
}

}  // namespace fk

static unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static void full_validate(const blr_problem* pb, int prec, const double* F, double dt,
                          const double* err_out) {
  require(pb != nullptr && F != nullptr && err_out != nullptr, "null argument");
  require(pb->nx >= 1, "nx must be >= 1");
  require(pb->x_hi > pb->x_lo, "x_hi must exceed x_lo");
  require(pb->f_left && pb->f_right, "null inflow function");
  require((pb->wall_left == 0 || pb->wall_left == 1) && (pb->wall_right == 0 || pb->wall_right == 1),
          "problem.wall_left / wall_right must be 0 (inflow) or 1 (diffusive wall)");
  require(prec == BLR_FP32 || prec == BLR_FP64, "bad precision");
  require(std::isfinite(dt) && dt >= 0.0, "dt must be finite and >= 0");
  const bool two_d = pb->ny >= 2;
  if (two_d) {
    require(pb->ny <= (1 << 20) && (long)pb->nx * pb->ny <= (1L << 22),
            "problem.ny must be <= 2^20 and nx * ny <= 2^22");
    require(pb->y_hi > pb->y_lo, "y_hi must exceed y_lo");
    require(pb->f_bottom && pb->f_top, "null boundary function of a y face");
    require((pb->wall_bottom == 0 || pb->wall_bottom == 1) &&
                (pb->wall_top == 0 || pb->wall_top == 1),
            "problem.wall_bottom / wall_top must be 0 (inflow) or 1 (diffusive wall)");
    require(pb->face_rows >= 0 && pb->face_rows <= 15, "problem.face_rows must be in [0, 15]");
  } else {
    require(pb->ny >= 0, "problem.ny must be >= 0");
    require(pb->face_rows == 0, "problem.face_rows: one-dimensional space takes one row per face");
  }
}

// The device work of one step; err_full (the L2 norm of the change) lands in
// the pinned read-back buffer, whose address is returned.
static double* full_enqueue(blr_ctx ctx, const blr_problem* pb, int prec, double* F, double dt) {
  const bool two_d = pb->ny >= 2;
  const DevTables& tb = get_tables(ctx, pb->v, prec);
  const HostTables& h = tb.h;
  hipStream_t s = ctx->stream;
  const int nx = pb->nx, ny = two_d ? pb->ny : 1, n = h.n;
  const long ncells = (long)nx * ny;
  const double dx = (pb->x_hi - pb->x_lo) / nx;
  const double dy = two_d ? (pb->y_hi - pb->y_lo) / ny : 1.0;
  const double dvd = std::pow(h.dv, h.d);
  const int plane = h.d == 3 ? h.N * h.N : h.N;
  const int stride1 = h.d == 3 ? h.N : 1;  // velocity axis 1 (along y)
  const int esz = prec == BLR_FP32 ? 4 : 8;
  // cells per collision call: with 2D velocity all of them up to 1024 (the
  // launches of a 32^2 grid are small, more cells per launch fill the chip);
  // with 3D velocity 64 (the fused pair kernels' basis limit)
  const int chunk = (int)std::min<long>(ncells, h.d == 2 ? kMaxSelfRows : fk::kChunk);
  double* Fn = (double*)ctx->buf("full.Fn", (size_t)ncells * n * sizeof(double));
  void* Q = ctx->buf("full.Q", (size_t)chunk * n * esz);
  float* F32 = prec == BLR_FP32 ? (float*)ctx->buf("full.F32", (size_t)chunk * n * sizeof(float))
                                : nullptr;
  const unsigned nbx = nblocks(n, 256);
  double* part = (double*)ctx->buf("full.part", (size_t)ncells * nbx * sizeof(double));
  double* err = (double*)ctx->buf("full.err", sizeof(double));
  // the obstacle (two-dimensional space): faces after the rectangle's
  const ObstacleHost oh = two_d ? obstacle_host(pb) : ObstacleHost{};
  require(!oh.any || pb->f_obstacle, "problem.solid marks a cell: f_obstacle is needed");
  Obs2 ob{nullptr, nullptr, nullptr, pb->f_obstacle, two_d ? 2 * (nx + ny) : 2, oh.nob};
  if (oh.any) {
    ob.face = (const int*)ctx->upload("full.ob.face", oh.face.data(), oh.face.size() * sizeof(int));
    ob.nbmap = (const int*)ctx->upload("full.ob.nb", oh.nbmap.data(), oh.nbmap.size() * sizeof(int));
    ob.solid = (const uint8_t*)ctx->upload("full.ob.solid", oh.solid.data(), oh.solid.size());
  }
  // rho_w from the cells next to the walls before any cell is updated
  const int nrho = two_d ? 2 * (nx + ny) + oh.nob : 2;
  double* rho = (double*)ctx->buf("full.rho", (size_t)nrho * sizeof(double));
  fk::Faces fc{{pb->f_left, pb->f_right, pb->f_bottom, pb->f_top}, pb->face_rows};
  if (two_d) {
    const int walls = pb->wall_left | (pb->wall_right << 1) | (pb->wall_bottom << 2) |
                      (pb->wall_top << 3);
    hipLaunchKernelGGL(fk::k_full_face_rho2d, dim3(nrho), dim3(1024), 0, s, F, nx, ny, n, fc,
                       walls, ob, h.L, h.dv, plane, stride1, h.N, rho);
  } else {
    hipLaunchKernelGGL(fk::k_full_wall_rho, dim3(2), dim3(1024), 0, s, F, nx, n, pb->f_left,
                       pb->f_right, pb->wall_left, pb->wall_right, h.L, h.dv, plane, rho);
  }
  BLR_CHECK_LAUNCH();
  for (long p0 = 0; p0 < ncells; p0 += chunk) {
    const int np = (int)std::min<long>(chunk, ncells - p0);
    const double* rows = F + p0 * n;
    if (prec == BLR_FP32) {
      hipLaunchKernelGGL(fk::k_cast_f32, dim3(nblocks((long)np * n, 256)), dim3(256), 0, s, rows,
                         (long)np * n, F32);
      BLR_CHECK_LAUNCH();
      collision_self(ctx, pb->v, BLR_FP32, F32, np, Q);
    } else {
      collision_self(ctx, pb->v, BLR_FP64, rows, np, Q);
    }
    timed_begin("full.update", (double)np * n * 8.0 * (3.0 + 1.0) + (double)np * n * esz, s);
    if (two_d) {
      if (prec == BLR_FP32)
        hipLaunchKernelGGL(fk::k_full_update2d<float>, dim3(nbx, np), dim3(256), 0, s, F, nx, ny,
                           n, p0, (const float*)Q, fc, ob, rho, dt, dx, dy, h.L, h.dv, plane,
                           stride1, h.N, Fn, part);
      else
        hipLaunchKernelGGL(fk::k_full_update2d<double>, dim3(nbx, np), dim3(256), 0, s, F, nx, ny,
                           n, p0, (const double*)Q, fc, ob, rho, dt, dx, dy, h.L, h.dv, plane,
                           stride1, h.N, Fn, part);
    } else if (prec == BLR_FP32) {
      hipLaunchKernelGGL(fk::k_full_update<float>, dim3(nbx, np), dim3(256), 0, s, F, nx, n,
                         (int)p0, (const float*)Q, pb->f_left, pb->f_right, rho, dt, dx, h.L,
                         h.dv, plane, Fn, part);
    } else {
      hipLaunchKernelGGL(fk::k_full_update<double>, dim3(nbx, np), dim3(256), 0, s, F, nx, n,
                         (int)p0, (const double*)Q, pb->f_left, pb->f_right, rho, dt, dx, h.L,
                         h.dv, plane, Fn, part);
    }
    BLR_CHECK_LAUNCH();
    timed_end(s);
  }
  hipLaunchKernelGGL(fk::k_err_total, dim3(1), dim3(256), 0, s, part, ncells * nbx, dx * dy * dvd,
                     err);
  BLR_CHECK_LAUNCH();
  BLR_HIP(hipMemcpyAsync(F, Fn, (size_t)ncells * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double* hb = (double*)ctx->host_readback(sizeof(double));
  BLR_HIP(hipMemcpyAsync(hb, err, sizeof(double), hipMemcpyDeviceToHost, s));
  return hb;
}

// One step.  Unless kernels are timed, the device work is recorded as a graph
// the second time a configuration (problem, F, dt, precision) is seen and
// replayed from then on: at 2D grids of 32^2 points the step is a thousand
// small launches, whose issue costs more than their work.
void full_step(blr_ctx ctx, const blr_problem* pb, int prec, double* F, double dt,
               double* err_out) {
  full_validate(pb, prec, F, dt, err_out);
  hipStream_t s = ctx->stream;
  auto eager = [&]() {
    double* hb = full_enqueue(ctx, pb, prec, F, dt);
    BLR_HIP(hipStreamSynchronize(s));
    *err_out = hb[0];
  };
  if (ctx->timer.on) {
    eager();
    return;
  }
  std::string key = "full#";
  key.append((const char*)pb, sizeof(*pb));
  key.append((const char*)&F, sizeof(F));
  key.append((const char*)&dt, sizeof(dt));
  key.append((const char*)&prec, sizeof(prec));
  if (pb->ny >= 2) {   // the mask's content (a host array read at every call)
    const uint64_t oh = obstacle_host(pb).hash;
    key.append((const char*)&oh, sizeof(oh));
  }
  auto& gs = ctx->graphs;
  size_t gi = gs.size();
  for (size_t k = 0; k < gs.size(); ++k)
    if (gs[k].key == key) gi = k;
  if (gi == gs.size()) {
    if (gs.size() >= 8) {  // forget the oldest
      if (gs.front().exec) (void)hipGraphExecDestroy(gs.front().exec);
      if (gs.front().exec2) (void)hipGraphExecDestroy(gs.front().exec2);
      gs.erase(gs.begin());
    }
    gs.push_back(blr_ctx_t::StepGraph{});
    gi = gs.size() - 1;
    gs[gi].key = key;
  }
  auto& g = gs[gi];
  if (g.gen != ctx->buf_gen) {  // addresses moved: start over
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.seen = 0;
    g.gen = ctx->buf_gen;
  }
  if (!g.exec && g.seen == 0) {
    eager();
    g.seen = 1;
    g.gen = ctx->buf_gen;
    return;
  }
  if (!g.exec) {
    if (!ctx->cap_stream) BLR_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const uint64_t gen0 = ctx->buf_gen;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    ctx->capture_broken = false;
    hipGraph_t graph = nullptr;
    double* hb = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        hb = full_enqueue(ctx, pb, prec, F, dt);
      } catch (...) {
        (void)hipStreamEndCapture(ctx->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        ctx->stream = s;
        ctx->capturing = false;
        (void)hipGetLastError();
        eager();  // the same kernels directly; an error of the step's own is reported there
        g.gen = ctx->buf_gen;
        return;
      }
      e = hipStreamEndCapture(ctx->cap_stream, &graph);
    }
    ctx->stream = s;
    ctx->capturing = false;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && graph && !ctx->capture_broken && ctx->buf_gen == gen0)
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || !exec) {
      (void)hipGetLastError();
      eager();  // not recordable this time: run it directly
      g.gen = ctx->buf_gen;
      return;
    }
    g.exec = exec;
    g.gen = ctx->buf_gen;
    g.hb = hb;
  }
  BLR_HIP(hipGraphLaunch(g.exec, s));
  BLR_HIP(hipStreamSynchronize(s));
  *err_out = g.hb[0];
}

}  // namespace blr

// ------------------------------------------------------------------ C ABI --
extern "C" blr_status blr_full_step(blr_ctx ctx, const blr_problem* pb, blr_precision prec,
                                    double* F, double dt, double* err_full) {
  if (!ctx) return BLR_ERR_ARG;
  ctx->err.clear();
  try {
    BLR_HIP(hipSetDevice(ctx->device));
    blr::full_step(ctx, pb, prec, F, dt, err_full);
    return BLR_OK;
  } catch (const blr::Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return BLR_ERR_HIP;
  }
}
