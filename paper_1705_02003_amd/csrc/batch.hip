// Batched ensemble PCG: many ensembles of different width, grid and
// iteration count advanced together, one CG step per graph replay.
//
// Every ensemble keeps its own matrix, vectors, per-member state and
// partial buffers (its ens_pcg_solve workspace).  One CG step for all
// ensembles is four launches: a fused stencil kernel and an update kernel,
// each on a fixed grid of G workgroups that stride over the work units of
// all ensembles (persistent style), and after each a finish kernel with one
// workgroup per ensemble.  The four launches form a hipGraph built once from
// kernel nodes and replayed until every ensemble has retired; an ensemble
// that has retired contributes no work.  A retiring ensemble stamps the
// device's constant-rate clock, which gives per-ensemble latencies.
//
// Work assignment: unit u (a tile of one ensemble, or a chunk of 2048
// elements for the update) goes to the workgroup with logical index
// L = u mod G; logical indices are laid out so that consecutive ones run on
// one XCD (workgroup ids are dispatched round-robin over the eight XCDs).
// The partial sums of ensemble e from logical workgroup L land in row
// (L - first_unit(e)) mod G, so row r always holds the units r, r + G, ... of
// that ensemble in that order: a fixed reduction tree, the same for every
// member.  The paper treats variable ensemble sizes as future work
// (Section 5); this is the batched form of the same solver.
#include <algorithm>
#include <cstring>
#include <vector>

#include "device.h"

namespace ens {

constexpr int kUpdateChunk = kNT * 2 * 4;  // elements per update unit (VEC 2, 4 strides)
constexpr int kGraphSteps = 16;            // CG steps per graph launch (at most)
constexpr int kMaxBatch = 1024;             // ensembles per batch (tables staged in LDS)

struct BatchEns {
  const double* V;
  const double* b;
  double* x;
  double* p[2];
  double* q;
  double* r;
  double* partial;
  Members m;
  int n, S, tpp;          // tpp: threads per point of the element-wise kernel (S / 2)
  int sw, stpp;           // member tile width and its threads per point (sw / 2)
  int tx, ty, nchunk, ntiles;   // ntiles: spatial tiles per member tile
  size_t nelem, vstride;
  int unit0;    // first stencil unit; units are (member tile, spatial tile)
  int eunit0;   // first update unit
  int neunits;  // update units
};

struct BatchArgs {
  const BatchEns* ens;
  const int* unit0;   // [n_ens + 1] prefix of stencil units
  const int* eunit0;  // [n_ens + 1] prefix of update units
  int* done;          // [n_ens]
  unsigned long long* clock;  // [1 + n_ens]: start, then retirement per ensemble
  int n_ens;
  int U, EU;
  int G;
  double rtol;
};

__device__ __forceinline__ int logical_group(int b, int G) {
  return (G >= 8 && (G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

// ensemble owning unit u: the largest e with prefix[e] <= u
__device__ __forceinline__ int owner(const int* prefix, int n, int u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A value that is the same in every lane (an ensemble's descriptor field):
// moving it to a scalar register right after its load keeps later address
// arithmetic off vector registers whose loads the compiler would otherwise
// wait for again at every branch merge.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ size_t uni(size_t v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((size_t)hi << 32) | lo;
}

template <class T>
__device__ __forceinline__ T* uni(T* p) {
  return reinterpret_cast<T*>(uni(reinterpret_cast<size_t>(p)));
}

// stage the unit prefix table and the retirement flags in LDS
__device__ __forceinline__ void stage_tables(const int* prefix, const int* done, int n, int* s_prefix,
                                             int* s_done) {
  for (int k = threadIdx.x; k <= n; k += kNT) s_prefix[k] = prefix[k];
  for (int k = threadIdx.x; k < n; k += kNT) s_done[k] = done[k];
  __syncthreads();
}

__device__ __forceinline__ int partial_row(int L, int first, int G) {
  int r = (L - first) % G;
  return r < 0 ? r + G : r;
}

template <bool SYM>
__global__ __launch_bounds__(kNT) void batch_stencil_kernel(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) double ring[4][kRing];
  __shared__ __attribute__((aligned(16))) double sym[SYM ? 6 * kRing : 2];
  __shared__ double red[kWaves * 64 * 2];
  __shared__ int s_prefix[kMaxBatch + 1];
  __shared__ int s_done[kMaxBatch];
  stage_tables(a.unit0, a.done, a.n_ens, s_prefix, s_done);
  const int t = threadIdx.x;
  const int L = logical_group(blockIdx.x, a.G);
  const double zero2[2] = {0.0, 0.0};
  int cur = -1, cur_js = 0, cur_first = 0, tpp = 1, S = 2, ntiles = 1;
  double* partial = nullptr;
  double beta[2] = {0.0, 0.0}, aprev[2] = {0.0, 0.0}, acc[2] = {0.0, 0.0}, acc2[2] = {0.0, 0.0};
  TileView tv = {};
  // rows of a member tile's partials: row r holds its units r, r + G, ...
  auto flush = [&]() {
    group_reduce<2>(acc, tpp, red);
    if (t < tpp) {
      const int row = partial_row(L, cur_first, a.G);
#pragma unroll
      for (int c = 0; c < 2; ++c) gstore(&partial[(size_t)row * S + tv.s0 + t * 2 + c], acc[c]);
    }
  };
  int e = 0;
  for (int u = L; u < a.U; u += a.G) {
    if (u >= s_prefix[e + 1]) e = owner(s_prefix, a.n_ens, u);   // next ensemble
    e = uni(e);
    if (uni(s_done[e])) continue;
    const int local = u - s_prefix[e];
    if (e != cur) ntiles = uni(a.ens[e].ntiles);
    const int js = local / ntiles;            // member tile
    const int first = s_prefix[e] + js * ntiles;
    if (e != cur || js != cur_js) {
      if (cur >= 0) flush();
      const BatchEns& E = a.ens[e];
      cur = e;
      cur_js = js;
      cur_first = first;
      S = uni(E.S);
      tpp = uni(E.stpp);
      partial = uni(E.partial);
      tv.s0 = js * uni(E.sw);
      const int sv = tv.s0 + (t % tpp) * 2;
      const int it = uni(gload(&E.m.ctl[CTL_K])) + 1;   // the iteration this launch performs
      double* const* pp = E.p;
      tv.V = uni(E.V);
      tv.r = uni(E.r);
      tv.pold = uni(pp[(it + 1) & 1]);
      tv.pnew = uni(pp[it & 1]);
      tv.q = uni(E.q);
      tv.x = uni(E.x);
      tv.n = uni(E.n);
      tv.S = S;
      tv.sw = uni(E.sw);
      tv.swp = tv.sw;   // power-of-two widths: every member tile is full
      tv.tpp = tpp;
      tv.tx = uni(E.tx);
      tv.ty = uni(E.ty);
      tv.nchunk = uni(E.nchunk);
      tv.nelem = uni(E.nelem);
      tv.vstride = uni(E.vstride);
      const double* mb = uni(E.m.beta);
      const double* ma = uni(E.m.alpha_prev);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        // consumed here (the select), once per member tile: a load still
        // pending at the unit loop's head would make each tile wait for the
        // previous tile's stores
        const double bt = gload(&mb[sv + c]);
        const double ap = gload(&ma[sv + c]);
        beta[c] = (sv + c < S) ? bt : 0.0;
        aprev[c] = (sv + c < S) ? ap : 0.0;
        acc[c] = 0.0;
      }
    }
    stencil_tile<2, M_PCG_J, SYM>(tv, local - js * ntiles, ring, sym, beta, aprev, zero2, zero2, acc,
                                  acc2);
  }
  if (cur >= 0) flush();
}

// r -= alpha q for members with a step (step[c] = alpha if the member is
// active, else 0), then the partial sums r^T r and r^T z (z = r / diag) of
// two members
__device__ __forceinline__ void update_pair(double (&rv)[2], const double (&qv)[2], const double (&dv)[2],
                                            const double (&step)[2], double (&rr)[2], double (&rz)[2]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (step[c] != 0.0) rv[c] = fma(-step[c], qv[c], rv[c]);
    rr[c] = fma(rv[c], rv[c], rr[c]);
    rz[c] = fma(rv[c], rv[c] / dv[c], rz[c]);
  }
}

__global__ __launch_bounds__(kNT) void batch_update_kernel(BatchArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  __shared__ int s_prefix[kMaxBatch + 1];
  __shared__ int s_done[kMaxBatch];
  stage_tables(a.eunit0, a.done, a.n_ens, s_prefix, s_done);
  const int t = threadIdx.x;
  const int L = logical_group(blockIdx.x, a.G);
  int cur = -1, tpp = 1, S = 2;
  double step[2] = {0.0, 0.0}, rz[2] = {0.0, 0.0}, rr[2] = {0.0, 0.0};
  int e = 0;
  const double* r_in = nullptr;
  double* r_out = nullptr;
  const double* q_in = nullptr;
  const double* d_in = nullptr;
  size_t nelem = 0;
  int first = 0, rows = 1;
  double* partial = nullptr;
  auto flush = [&]() {
    group_reduce<2>(rr, tpp, red);
    group_reduce<2>(rz, tpp, red);
    if (t < tpp) {
      const int row = partial_row(L, first, a.G);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        gstore(&partial[(size_t)row * S + t * 2 + c], rz[c]);
        gstore(&partial[(size_t)rows * S + (size_t)row * S + t * 2 + c], rr[c]);
      }
    }
  };
  for (int u = L; u < a.EU; u += a.G) {
    if (u >= s_prefix[e + 1]) e = owner(s_prefix, a.n_ens, u);   // next ensemble
    e = uni(e);
    if (uni(s_done[e])) continue;
    if (e != cur) {
      if (cur >= 0) flush();
      cur = e;
      const BatchEns& E = a.ens[e];
      S = uni(E.S);
      tpp = uni(E.tpp);
      nelem = uni(E.nelem);
      first = s_prefix[e];
      rows = min(a.G, uni(E.neunits));
      partial = uni(E.partial);
      r_in = uni(E.r);
      r_out = uni(E.r);
      q_in = uni(E.q);
      d_in = uni(E.V) + 4 * uni(E.vstride);
      const int sv = (t % tpp) * 2;
      const int* ma = uni(E.m.active);
      const double* mal = uni(E.m.alpha);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        // consumed here, once per ensemble: a load still pending at the
        // unit loop's head would make every unit wait for the previous
        // unit's stores
        const int on = gload(&ma[sv + c]);
        const double al = gload(&mal[sv + c]);
        step[c] = on ? al : 0.0;
        rz[c] = 0.0;
        rr[c] = 0.0;
      }
    }
    const size_t base = (size_t)(u - first) * kUpdateChunk;
    if (base + kUpdateChunk <= nelem) {
      // a whole chunk: twelve loads in flight, no per-lane predicates
      double rv[4][2], qv[4][2], dv[4][2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t el = base + ((size_t)k * kNT + t) * 2;
        ld<2>(rv[k], r_in + el);
        ld<2>(qv[k], q_in + el);
        ld<2>(dv[k], d_in + el);
      }
      // keep the scheduler from starting the arithmetic (and its waits)
      // before all twelve loads are issued
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        update_pair(rv[k], qv[k], dv[k], step, rr, rz);
        st<2>(r_out + base + ((size_t)k * kNT + t) * 2, rv[k]);
      }
    } else {
      // the ensemble's last, partial chunk
      for (int k = 0; k < 4; ++k) {
        const size_t el = base + ((size_t)k * kNT + t) * 2;
        if (el < nelem) {
          double rv[2], qv[2], dv[2];
          ld<2>(rv, r_in + el);
          ld<2>(qv, q_in + el);
          ld<2>(dv, d_in + el);
          update_pair(rv, qv, dv, step, rr, rz);
          st<2>(r_out + el, rv);
        }
      }
    }
  }
  if (cur >= 0) flush();
}

// one workgroup per ensemble: alpha (stage 0) or the convergence test and
// beta (stage 1), which retires the ensemble when its last member stops
template <int STAGE>
__global__ __launch_bounds__(kFinNT) void batch_finish_kernel(BatchArgs a) {
  __shared__ double fin[2 * kFinNT * 2];
  __shared__ int live;
  const int e = blockIdx.x;
  if (a.done[e]) return;
  const BatchEns& E = a.ens[e];
  if (gload(&E.m.ctl[CTL_DONE])) {
    // retired before the first step (every member had b = 0)
    if (STAGE == 0 && threadIdx.x == 0) {
      a.clock[1 + e] = wall_clock64();
      a.done[e] = 1;
    }
    return;
  }
  FinishArgs f = {};
  f.partial = E.partial;
  f.m = E.m;
  f.g.S = E.S;
  f.g.Sp = E.S;
  f.g.vec = 2;
  f.rtol = a.rtol;
  if (STAGE == 0) {
    f.kind = F_ALPHA;
    f.G = min(a.G, E.ntiles);
    (void)finish_body<2>(f, fin, live);
  } else {
    f.kind = F_UPDATE_J;
    f.G = min(a.G, E.neunits);
    const int retired = finish_body<2>(f, fin, live);
    if (retired && threadIdx.x == 0) {
      a.clock[1 + e] = wall_clock64();
      a.done[e] = 1;
    }
  }
}

__global__ void batch_stamp_kernel(unsigned long long* clock) {
  if (threadIdx.x == 0) clock[0] = wall_clock64();
}

}  // namespace ens

using namespace ens;

namespace {

size_t align256b(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
  BatchEns* ens;
  int* unit0;
  int* eunit0;
  int* done;
  unsigned long long* clock;
  size_t bytes;
};

BatchLayout batch_layout(void* base, int n) {
  BatchLayout l;
  char* p = static_cast<char*>(base);
  size_t off = 0;
  l.ens = reinterpret_cast<BatchEns*>(p + off);
  off += align256b(sizeof(BatchEns) * (size_t)n);
  l.unit0 = reinterpret_cast<int*>(p + off);
  off += align256b(sizeof(int) * (size_t)(n + 1));
  l.eunit0 = reinterpret_cast<int*>(p + off);
  off += align256b(sizeof(int) * (size_t)(n + 1));
  l.done = reinterpret_cast<int*>(p + off);
  off += align256b(sizeof(int) * (size_t)n);
  l.clock = reinterpret_cast<unsigned long long*>(p + off);
  off += align256b(sizeof(unsigned long long) * (size_t)(n + 1));
  l.bytes = off;
  return l;
}

int hip_fail(hipError_t e) { return set_hip_error(e); }

}  // namespace

extern "C" {

size_t ens_batch_workspace_bytes(int32_t n_items) {
  if (n_items < 1 || n_items > kMaxBatch) return 0;
  return batch_layout(nullptr, n_items).bytes;
}

int ens_batch_solve(const ens_opts* opts, int32_t n_items, ens_batch_item* items, void* batch_ws,
                    size_t batch_ws_bytes, void* stream) {
  if (n_items < 1 || n_items > kMaxBatch || !items || !batch_ws) return ENS_EINVAL;
  if (batch_ws_bytes < ens_batch_workspace_bytes(n_items)) return ENS_ENOMEM;
  ens_opts o0;
  std::memset(&o0, 0, sizeof(o0));
  const ens_opts* o = opts ? opts : &o0;
  if (o->precond != ENS_PRECOND_JACOBI) return ENS_ENOTSUP;
  const double rtol = (o->rtol != 0.0) ? o->rtol : 1e-8;
  const int max_iter = o->max_iter ? o->max_iter : 20000;
  const int poll = o->poll_every ? o->poll_every : 16;
  const int G = std::min(kMaxGroups, o->max_groups ? o->max_groups : 512) & ~7;
  if (!(rtol >= 0.0) || max_iter < 1 || poll < 1 || G < 8) return ENS_EINVAL;
  for (int k = 0; k < n_items; ++k) {
    const ens_batch_item& it = items[k];
    const int S = it.S;
    if (it.prob.dim == 3) return ENS_ENOTSUP;
    if (it.prob.n < 2 || it.prob.n > 16384 || !valid_S(S)) return ENS_EINVAL;
    if (S < 2 || (S & (S - 1)) != 0) return ENS_ENOTSUP;   // batched widths: powers of two
    if (!it.V_dev || !it.b_dev || !it.x_dev || !it.ws_dev || it.tile_lines < 0) return ENS_EINVAL;
    if (it.member_tile < 0 || (it.member_tile & (it.member_tile - 1)) != 0) return ENS_EINVAL;
    const size_t nr = (size_t)it.prob.n * it.prob.n;
    if (it.ws_bytes < workspace_bytes(nr, S, false)) return ENS_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  const BatchLayout lay = batch_layout(batch_ws, n_items);

  // per-ensemble set-up: r = b, x = 0, p_0 = 0, ||b||, rho, masks
  std::vector<BatchEns> host(n_items);
  std::vector<int> u0(n_items + 1), e0(n_items + 1);
  std::vector<Geometry> geo(n_items);
  u0[0] = e0[0] = 0;
  for (int k = 0; k < n_items; ++k) {
    const ens_batch_item& it = items[k];
    Geometry g = make_geometry(it.prob.n, it.S, it.tile_lines, G, it.member_tile);
    geo[k] = g;
    char* base = static_cast<char*>(it.ws_dev);
    // same carve as ens_pcg_solve (Jacobi layout)
    Workspace w = carve_workspace(base, (size_t)it.prob.n * it.prob.n, it.S, false);
    hipError_t he = hipMemsetAsync(w.m.ctl, 0, sizeof(int) * CTL_COUNT, s);
    if (he != hipSuccess) return hip_fail(he);
    InitArgs ia;
    std::memset(&ia, 0, sizeof(ia));
    ia.V = it.V_dev;
    ia.b = it.b_dev;
    ia.x = it.x_dev;
    ia.p0 = w.p[0];
    ia.r = w.r;
    ia.partial = w.partial;
    ia.m = w.m;
    ia.g = g;
    ia.max_iter = max_iter;
    const int ge = init_groups(g);
    launch_init(ia, ge, s);
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = ge;
    f.kind = F_INIT;
    f.m = w.m;
    f.g = g;
    f.max_iter = max_iter;
    launch_finish(f, s);
    BatchEns& E = host[k];
    std::memset(&E, 0, sizeof(E));
    E.V = it.V_dev;
    E.b = it.b_dev;
    E.x = it.x_dev;
    E.p[0] = w.p[0];
    E.p[1] = w.p[1];
    E.q = w.q;
    E.r = w.r;
    E.partial = w.partial;
    E.m = w.m;
    E.n = g.n;
    E.S = g.S;
    E.tpp = g.tpp;
    E.sw = g.sw;
    E.stpp = g.stpp;
    E.tx = g.tx;
    E.ty = g.ty;
    E.nchunk = g.nchunk;
    E.ntiles = g.ntiles;
    E.nelem = g.nelem;
    E.vstride = g.vstride;
    E.unit0 = u0[k];
    E.eunit0 = e0[k];
    E.neunits = (int)((g.nelem + kUpdateChunk - 1) / kUpdateChunk);
    u0[k + 1] = u0[k] + g.nstile * g.ntiles;
    e0[k + 1] = e0[k] + E.neunits;
  }
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = hipMemcpyAsync(lay.ens, host.data(), sizeof(BatchEns) * n_items, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(lay.unit0, u0.data(), sizeof(int) * (n_items + 1), hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemcpyAsync(lay.eunit0, e0.data(), sizeof(int) * (n_items + 1), hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipMemsetAsync(lay.done, 0, sizeof(int) * n_items, s);
  if (he == hipSuccess) he = hipMemsetAsync(lay.clock, 0, sizeof(unsigned long long) * (n_items + 1), s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);   // host tables consumed
  if (he != hipSuccess) return hip_fail(he);

  BatchArgs ba;
  ba.ens = lay.ens;
  ba.unit0 = lay.unit0;
  ba.eunit0 = lay.eunit0;
  ba.done = lay.done;
  ba.clock = lay.clock;
  ba.n_ens = n_items;
  ba.U = u0[n_items];
  ba.EU = e0[n_items];
  ba.G = G;
  ba.rtol = rtol;

  // CG steps for every ensemble: a graph of `steps` x four kernel nodes.
  // Several steps per graph launch amortise the few microseconds between
  // consecutive graph executions; steps after an ensemble retires find its
  // done flag and return at once.
  const int steps = std::min(poll, kGraphSteps);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  he = hipGraphCreate(&graph, 0);
  void* args[1] = {&ba};
  hipGraphNode_t prev = nullptr;
  const void* stencil_fn = (o->flags & ENS_FLAG_FULL_STENCIL)
                               ? reinterpret_cast<const void*>(&batch_stencil_kernel<false>)
                               : reinterpret_cast<const void*>(&batch_stencil_kernel<true>);
  struct NodeSpec {
    const void* fn;
    unsigned grid, block;
  } specs[4] = {{stencil_fn, (unsigned)G, (unsigned)kNT},
                {reinterpret_cast<const void*>(&batch_finish_kernel<0>), (unsigned)n_items, (unsigned)kFinNT},
                {reinterpret_cast<const void*>(&batch_update_kernel), (unsigned)G, (unsigned)kNT},
                {reinterpret_cast<const void*>(&batch_finish_kernel<1>), (unsigned)n_items, (unsigned)kFinNT}};
  for (int k = 0; k < 4 * steps && he == hipSuccess; ++k) {
    const NodeSpec& sp = specs[k % 4];
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void*>(sp.fn);
    kp.gridDim = dim3(sp.grid);
    kp.blockDim = dim3(sp.block);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    he = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  int32_t* flags = nullptr;
  if (he == hipSuccess) he = hipHostMalloc((void**)&flags, 2 * sizeof(int32_t) * n_items, hipHostMallocDefault);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (int k = 0; k < 2 && he == hipSuccess; ++k) he = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
  if (he == hipSuccess) {
    hipLaunchKernelGGL(batch_stamp_kernel, dim3(1), dim3(64), 0, s, lay.clock);
    he = hipGetLastError();
  }
  int launched = 0, slot = 0;
  bool have_prev = false;
  while (he == hipSuccess && launched < max_iter) {
    const int chunk = std::min(poll, max_iter - launched);
    for (int c = 0; c < chunk && he == hipSuccess; c += steps) he = hipGraphLaunch(exec, s);
    launched += chunk;
    if (he != hipSuccess) break;
    int32_t* f = flags + slot * n_items;
    he = hipMemcpyAsync(f, lay.done, sizeof(int32_t) * n_items, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipEventRecord(ev[slot], s);
    if (he == hipSuccess && have_prev) {
      he = hipEventSynchronize(ev[slot ^ 1]);
      if (he == hipSuccess) {
        const int32_t* pf = flags + (slot ^ 1) * n_items;
        bool all = true;
        for (int k = 0; k < n_items; ++k) all = all && pf[k];
        if (all) break;
      }
    }
    have_prev = true;
    slot ^= 1;
  }
  int rc = (he == hipSuccess) ? ENS_OK : hip_fail(he);

  // deferred x update of each ensemble's last iteration, then results
  std::vector<unsigned long long> clk(n_items + 1, 0);
  if (rc == ENS_OK) {
    for (int k = 0; k < n_items; ++k)
      launch_final(items[k].x_dev, host[k].p[0], host[k].p[1], host[k].m, geo[k], init_groups(geo[k]), s);
    he = hipGetLastError();
    if (he == hipSuccess) he = hipMemcpyAsync(clk.data(), lay.clock, sizeof(unsigned long long) * (n_items + 1),
                                              hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) rc = hip_fail(he);
  }
  int rate_khz = 0;
  if (rc == ENS_OK) {
    int dev = 0;
    he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    if (he != hipSuccess) rc = hip_fail(he);
  }
  for (int k = 0; k < n_items && rc == ENS_OK; ++k) {
    ens_batch_item& it = items[k];
    const int S = it.S;
    int32_t iters[kMaxS], status[kMaxS];
    double relres[kMaxS];
    he = hipMemcpy(iters, host[k].m.iters, sizeof(int32_t) * S, hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipMemcpy(status, host[k].m.status, sizeof(int32_t) * S, hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipMemcpy(relres, host[k].m.relres, sizeof(double) * S, hipMemcpyDeviceToHost);
    if (he != hipSuccess) {
      rc = hip_fail(he);
      break;
    }
    int ei = 0;
    for (int q = 0; q < S; ++q) ei = std::max(ei, (int)iters[q]);
    it.ens_iters = ei;
    if (it.iters_host) std::memcpy(it.iters_host, iters, sizeof(int32_t) * S);
    if (it.status_host) std::memcpy(it.status_host, status, sizeof(int32_t) * S);
    if (it.relres_host) std::memcpy(it.relres_host, relres, sizeof(double) * S);
    const unsigned long long c1 = clk[1 + k] ? clk[1 + k] : clk[0];
    it.seconds = (rate_khz > 0 && c1 >= clk[0]) ? (double)(c1 - clk[0]) / ((double)rate_khz * 1e3) : 0.0;
  }
  for (int k = 0; k < 2; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  if (flags) (void)hipHostFree(flags);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  return rc;
}

}  // extern "C"
