// C ABI of libens: argument validation, workspace carving and the host loop
// that drives the ensemble PCG kernels.  See include/ens.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "fe3d.h"
#include "multigrid.h"

namespace ens {

static thread_local int g_last_hip_error = 0;

int set_hip_error(hipError_t e) {
  g_last_hip_error = (int)e;
  return ENS_EHIP;
}

int valid_S(int S) { return S >= 1 && S <= kMaxS; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: a small header (partials, per-member state, control words)
// followed by the ensemble vectors.
static size_t header_bytes() {
  size_t b = 0;
  b += align256(sizeof(double) * (size_t)kMaxS * 16);              // staged parameters
  b += align256(sizeof(double) * 3 * (size_t)kMaxGroups * kMaxS);  // partials
  b += align256(sizeof(double) * 7 * (size_t)kMaxS);               // doubles
  b += align256(sizeof(double) * (size_t)kMaxS * kChebCoef);       // cheb
  b += align256(sizeof(double) * (size_t)kMaxS * 16);              // result
  b += align256(sizeof(int) * 3 * (size_t)kMaxS);                  // ints
  b += align256(sizeof(int) * CTL_COUNT);                          // control
  return b;
}

static int n_vectors(bool cheb) { return cheb ? 7 : 5; }

// bytes from one workspace vector to the next (see slot_stride)
static size_t vector_bytes(size_t nr, int S) { return sizeof(double) * slot_stride(nr * S); }

size_t workspace_bytes(size_t nr, int S, bool cheb) {
  return header_bytes() + vector_bytes(nr, S) * n_vectors(cheb);
}

Workspace carve_workspace(void* base, size_t nr, int S, bool cheb) {
  Workspace w;
  std::memset(&w, 0, sizeof(w));
  char* p = static_cast<char*>(base);
  w.y = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * (size_t)kMaxS * 16);
  w.partial = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * 3 * (size_t)kMaxGroups * kMaxS);
  double* dd = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * 7 * (size_t)kMaxS);
  w.m.rho = dd;
  w.m.alpha = dd + kMaxS;
  w.m.alpha_prev = dd + 2 * kMaxS;
  w.m.beta = dd + 3 * kMaxS;
  w.m.bnorm = dd + 4 * kMaxS;
  w.m.relres = dd + 5 * kMaxS;
  w.m.lmax = dd + 6 * kMaxS;
  w.m.cheb = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * (size_t)kMaxS * kChebCoef);
  w.m.result = reinterpret_cast<double*>(p);
  p += align256(sizeof(double) * (size_t)kMaxS * 16);
  int* ii = reinterpret_cast<int*>(p);
  p += align256(sizeof(int) * 3 * (size_t)kMaxS);
  w.m.active = ii;
  w.m.iters = ii + kMaxS;
  w.m.status = ii + 2 * kMaxS;
  w.m.ctl = reinterpret_cast<int*>(p);
  p += align256(sizeof(int) * CTL_COUNT);
  if (nr > 0) {
    const size_t vec = vector_bytes(nr, S);
    double** slots[7] = {&w.p[0], &w.p[1], &w.q, &w.r, &w.aux, &w.z[0], &w.z[1]};
    for (int k = 0; k < n_vectors(cheb); ++k) {
      *slots[k] = reinterpret_cast<double*>(p);
      p += vec;
    }
  }
  return w;
}

// Member lanes of an ensemble of S: VEC = 2 for even S, the slots of a point
// rounded up to a power of two.
static void member_lanes(Geometry& g, int S) {
  g.S = S;
  g.vec = (S % 2 == 0) ? 2 : 1;
  g.tpp = pow2ceil(S / g.vec);
  g.Sp = g.tpp * g.vec;
}

Geometry make_geometry(int n, int S, int tile_lines, int max_groups, int member_tile) {
  Geometry g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  member_lanes(g, S);
  // member tile: a power of two (the whole ensemble when it is at least S),
  // at least one thread's members wide; the last tile may hold fewer
  int sw = (member_tile > 0 && member_tile < S) ? member_tile : S;
  if (sw < g.vec) sw = g.vec;
  g.sw = sw;
  g.nstile = (S + sw - 1) / sw;
  g.stpp = (sw == S) ? g.tpp : pow2ceil(sw / g.vec);
  g.swp = g.stpp * g.vec;
  g.tx = kNT * g.vec / g.swp;
  g.nchunk = (n + g.tx - 1) / g.tx;
  // Defaults measured on MI355X at 512^2 and S = 1..64: 512 workgroups (two
  // per CU) with the tallest tile of at most 32 lines that still gives every
  // workgroup a tile.
  int G = (max_groups > 0) ? max_groups : 512;
  int ty = tile_lines;
  if (ty <= 0) {
    ty = 32;
    while (ty > 1 && (long long)g.nchunk * ((n + ty - 1) / ty) < G) ty >>= 1;
  }
  g.ty = std::min(ty, n);
  g.nband = (n + g.ty - 1) / g.ty;
  g.ntiles = g.nchunk * g.nband;
  G = std::min(std::min(G, g.ntiles), kMaxGroups);
  if (G >= 8) G &= ~7;
  g.groups = std::max(G, 1);
  g.nr = (size_t)n * n;
  g.nelem = g.nr * S;
  g.vstride = slot_stride(g.nelem);
  g.full = 0;
  g.dim = 2;
  g.nslot = 9;
  g.cslot = 4;
  return g;
}

// 3-D model: no tiles; the product kernel strides over pairs of points,
// kNT / tpp pairs per workgroup and pass, with at most 512 workgroups (two
// per CU, which its register use allows; at 31^3 points and S = 32 on
// MI355X the paired kernel at 512 workgroups is 5 % faster than one point
// per thread at 1024, and keeps the finishing kernels' partials half as
// large).
Geometry make_geometry3(int m, int S) {
  Geometry g;
  std::memset(&g, 0, sizeof(g));
  g.n = m;
  member_lanes(g, S);
  g.sw = S;
  g.nstile = 1;
  g.stpp = g.tpp;
  g.swp = g.Sp;
  g.nr = (size_t)m * m * m;
  g.nelem = g.nr * S;
  g.vstride = slot_stride(g.nelem);
  g.full = 1;
  g.dim = 3;
  g.nslot = 27;
  g.cslot = 13;
  // The product kernel takes g.np x-neighbouring points per thread: pairs
  // (a third fewer loads of p per point) when they give at least half the
  // 256 CUs a workgroup, single points on grids too small for that (coarse
  // multigrid levels, an S = 1 solve), which doubles the workgroups.  (At
  // 31^3, S = 8 pairs give 241 workgroups and single points were 2-4 %
  // slower; at 15^3, S = 32 pairs give 113 and single points were 25 %
  // faster.)
  const size_t ppb = (size_t)(kNT / g.tpp);
  const size_t npair = (size_t)((m + kFe3dPair - 1) / kFe3dPair) * m * m;
  size_t need = (npair + ppb - 1) / ppb;
  g.np = kFe3dPair;
  if (need < 128) {
    g.np = 1;
    need = (g.nr + ppb - 1) / ppb;
  }
  g.groups = (int)std::min<size_t>(need, 512);
  return g;
}

int init_groups(const Geometry& g) {
  const size_t per = (size_t)(kNT / g.tpp);   // points per workgroup and pass
  const size_t need = (g.nr + per - 1) / per;
  return (int)std::min<size_t>(std::max<size_t>(need, 1), 512);
}

static bool is3d(const ens_problem* p) { return p->dim == 3; }

static int check_problem(const ens_problem* p) {
  if (!p) return ENS_EINVAL;
  if (is3d(p)) {
    if (p->n < 2 || p->n > 1024) return ENS_EINVAL;
    if (p->d < 1 || p->d > kMaxTerms) return ENS_EINVAL;
    if ((p->eps_model != 0 && p->eps_model != 1) || p->amp != 0.0) return ENS_EINVAL;
    return ENS_OK;
  }
  if (p->dim != 0 && p->dim != 2) return ENS_EINVAL;
  if (p->n < 2 || p->n > 16384) return ENS_EINVAL;
  if (p->d < 2 || p->d > 16) return ENS_EINVAL;
  if (p->eps_model != 0 && p->eps_model != 1) return ENS_EINVAL;
  if (!std::isfinite(p->amp) || std::fabs(p->amp) >= 1.0) return ENS_EINVAL;
  return ENS_OK;
}

static size_t rows_of(const ens_problem* p) {
  const size_t n = (size_t)p->n;
  return is3d(p) ? n * n * n : n * n;
}

struct Opts {
  int precond, degree, max_iter, poll, tile_lines, max_groups, flags, member_tile;
  double ratio, rtol;
};

static int resolve_opts(const ens_opts* o, Opts& r) {
  ens_opts z;
  std::memset(&z, 0, sizeof(z));
  if (!o) o = &z;
  r.precond = o->precond;
  r.degree = o->cheb_degree ? o->cheb_degree : 4;
  r.ratio = (o->cheb_ratio != 0.0) ? o->cheb_ratio : 30.0;
  r.rtol = (o->rtol != 0.0) ? o->rtol : 1e-8;
  r.max_iter = o->max_iter ? o->max_iter : 20000;
  r.poll = o->poll_every;   // 0: adaptive (poll_interval)
  r.tile_lines = o->tile_lines;
  r.max_groups = o->max_groups;
  r.flags = o->flags;
  r.member_tile = o->member_tile;
  if (r.precond != ENS_PRECOND_JACOBI && r.precond != ENS_PRECOND_CHEBYSHEV &&
      r.precond != ENS_PRECOND_MULTIGRID)
    return ENS_EINVAL;
  if (r.precond == ENS_PRECOND_MULTIGRID) r.degree = kMgDegree;
  if (r.degree < 2 || r.degree > kMaxCheb) return ENS_EINVAL;
  if (!std::isfinite(r.ratio) || r.ratio <= 1.0) return ENS_EINVAL;
  if (!std::isfinite(r.rtol) || r.rtol < 0.0) return ENS_EINVAL;
  if (r.max_iter < 1 || r.poll < 0 || r.tile_lines < 0 || r.max_groups < 0) return ENS_EINVAL;
  if (r.member_tile < 0 || (r.member_tile & (r.member_tile - 1)) != 0 || r.member_tile > kMaxS)
    return ENS_EINVAL;
  return ENS_OK;
}

#define HIPCHECK(call)                       \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return set_hip_error(e_); \
  } while (0)

// A solve's workspace: the Krylov vectors and per-member state (8 vectors
// with a polynomial or multigrid preconditioner, 5 with Jacobi) and, for
// multigrid, the coarse levels after them.
static bool uses_poly(const Opts& o) { return o.precond != ENS_PRECOND_JACOBI; }

static int check_precond(const ens_problem* prob, const Opts& o) {
  if (o.precond != ENS_PRECOND_MULTIGRID) return ENS_OK;
  int ms[kMgMaxLevels];
  return (is3d(prob) && mg_levels(prob->n, ms) >= 2) ? ENS_OK : ENS_ENOTSUP;
}

static size_t solve_bytes(const ens_problem* prob, const Opts& o, int S) {
  size_t b = workspace_bytes(rows_of(prob), S, uses_poly(o));
  if (o.precond == ENS_PRECOND_MULTIGRID) b += mg_bytes(prob->n, S);
  return b;
}

static Workspace carve_solve(void* base, const ens_problem* prob, const Opts& o, int S, MgHierarchy* H) {
  const Workspace w = carve_workspace(base, rows_of(prob), S, uses_poly(o));
  if (H) {
    std::memset(H, 0, sizeof(*H));
    if (o.precond == ENS_PRECOND_MULTIGRID)
      mg_carve(static_cast<char*>(base) + workspace_bytes(rows_of(prob), S, true), prob->n, S, w.m.ctl, *H);
  }
  return w;
}

static void finish(const Workspace& w, const Geometry& g, int G, int kind, hipStream_t s,
                   double rtol = 0.0, int cheb_init = 0) {
  FinishArgs f;
  std::memset(&f, 0, sizeof(f));
  f.partial = w.partial;
  f.G = G;
  f.kind = kind;
  f.m = w.m;
  f.g = g;
  f.rtol = rtol;
  f.cheb_init = cheb_init;
  launch_finish(f, s);
}

// One preconditioner application z = p(D^-1 A) D^-1 r: the start step
// z_0 = D^-1 r / theta (already done by the caller when `started`), then
// degree-1 stencil steps; z_k is in w.z[k & 1].  The steps form the
// increment from the iterates (no vector of it is kept), from the third step
// on reading z_{k-2} from the buffer that z_k then overwrites.  Returns the
// buffer holding z.
static double* cheb_apply(const double* V, const Workspace& w, const Geometry& g, int degree,
                          bool init, bool started, hipStream_t s, const double* r = nullptr,
                          int first_step = 1) {
  if (!r) r = w.r;
  if (!started) launch_cheb_start(V, r, w.z[0], w.m, g, init_groups(g), s);
  for (int k = first_step; k < degree; ++k) {
    StencilArgs a;
    std::memset(&a, 0, sizeof(a));
    a.V = V;
    a.r = r;
    a.src = w.z[(k - 1) & 1];
    a.zout = w.z[k & 1];
    a.zprev = k >= 3 ? w.z[k & 1] : nullptr;
    a.partial = w.partial;
    a.m = w.m;
    a.g = g;
    a.cheb_step = k;
    a.cheb_last = (k == degree - 1);
    a.cheb_init = init ? 1 : 0;
    launch_stencil<M_CHEB>(a, s);
  }
  finish(w, g, g.groups, F_CHEB, s, 0.0, init ? 1 : 0);
  return w.z[(degree - 1) & 1];
}

static Geometry geometry_for(const ens_problem* prob, const Opts& o, int S) {
  if (is3d(prob)) {
    Geometry g = make_geometry3(prob->n, S);
    g.full = (o.flags & ENS_FLAG_FULL_STENCIL) ? 1 : 0;
    if (o.max_groups > 0) g.groups = std::min(g.groups, o.max_groups);
    return g;
  }
  Geometry g = make_geometry(prob->n, S, o.tile_lines, o.max_groups, o.member_tile);
  g.full = (o.flags & ENS_FLAG_FULL_STENCIL) ? 1 : 0;
  return g;
}

// ------------------------------------------------------------ multigrid
// Level 0 of the V-cycle works in the solve's own vectors: its right-hand
// side is the PCG residual r, its output z[1] (the direction source of the
// next step), its smoother start z[0] (written by the residual update) and
// its residual aux.  Its smoother coefficients are the solve's (the
// initialisation computes them with degree 2).
static void mg_bind_fine(MgHierarchy& H, const double* V, const Workspace& w, const Geometry& g) {
  MgLevel& f = H.lv[0];
  f.g = g;
  f.V = V;
  f.b = w.r;
  f.x = w.z[1];
  f.res = w.aux;
  f.za = w.z[0];
  f.mem = w.m;
}

// Coarse operators (Galerkin products, level by level) and each coarse
// level's smoother bound and coefficients.
static void mg_setup(const MgHierarchy& H, const Workspace& w, double ratio, hipStream_t s) {
  for (int l = 0; l + 1 < H.L; ++l) {
    const MgLevel& f = H.lv[l];
    const MgLevel& c = H.lv[l + 1];
    MgRapArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.Vf = f.V;
    ra.Vc = const_cast<double*>(c.V);
    ra.mc = c.m;
    ra.S = c.g.S;
    ra.Sp = c.g.Sp;
    ra.nrc = c.g.nr;
    ra.vstride_f = f.g.vstride;
    ra.vstride_c = c.g.vstride;
    launch_mg_rap(ra, s);
    if (!H.levelwise && c.Vt) launch_mg_pack(c.V, c.g.vstride, c.Vt, c.m, c.g.S, s);
    MgGershArgs ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.V = c.V;
    ga.partial = w.partial;
    ga.S = c.g.S;
    ga.Sp = c.g.Sp;
    ga.nr = c.g.nr;
    ga.vstride = c.g.vstride;
    const int G = mg_groups(c.g.nr, c.g.Sp);
    launch_mg_gersh(ga, G, s);
    MgCoefArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.partial = w.partial;
    ca.G = G;
    ca.S = c.g.S;
    ca.Sp = c.g.Sp;
    ca.ratio = ratio;
    ca.lmax = c.mem.lmax;
    ca.cheb = c.mem.cheb;
    launch_mg_coef(ca, s);
  }
}

// x_l = V_l(b_l) for a level above the coarsest, whose pre-smoother start
// za is in place: pre-smoothing, residual, restriction (starting the
// next level's smoother, or solving the one-node coarsest level), the
// coarse cycle, prolongation, the residual with the post-smoother's start,
// and post-smoothing with its result added to x in place (on level 0 with
// the partial sums of dotv^T x into `partial`).
static void mg_cycle(const MgHierarchy& H, int l, hipStream_t s, const double* dotv = nullptr,
                     double* partial = nullptr) {
  const MgLevel& v = H.lv[l];
  const MgLevel& c = H.lv[l + 1];
  const int* done = v.mem.ctl + CTL_DONE;
  StencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = v.V;
  a.m = v.mem;
  a.g = v.g;
  a.r = v.b;
  a.src = v.za;
  a.zout = v.x;
  a.cheb_step = 1;
  launch_fe3d<M_CHEB>(a, s);
  std::memset(&a, 0, sizeof(a));
  a.V = v.V;
  a.m = v.mem;
  a.g = v.g;
  a.r = v.b;
  a.src = v.x;
  a.q = v.res;
  launch_fe3d<M_RESID>(a, s);
  // the coarse tail (levels of at most 7^3 nodes, down to the one-node
  // level) in one launch, unless the next level is already the last
  const bool tail = !H.levelwise && c.m <= kMgTailNodes && l + 2 < H.L && H.L - (l + 1) <= kMgTailLevels;
  MgTransferArgs t;
  std::memset(&t, 0, sizeof(t));
  t.fine_in = v.res;
  t.coarse_out = const_cast<double*>(c.b);
  t.Vc = c.V;
  t.cheb = c.mem.cheb;
  t.z = c.za;
  t.x = c.x;
  t.done = done;
  t.op = tail ? MG_RESTRICT : ((l + 2 == H.L) ? MG_RESTRICT_SOLVE : MG_RESTRICT_START);
  t.mc = c.m;
  t.S = c.g.S;
  t.Sp = c.g.Sp;
  t.vstride_c = c.g.vstride;
  launch_mg_transfer(t, s);
  if (tail) {
    MgTailArgs ta;
    std::memset(&ta, 0, sizeof(ta));
    ta.nlev = H.L - (l + 1);
    for (int j = 0; j < ta.nlev; ++j) {
      const MgLevel& q = H.lv[l + 1 + j];
      ta.lv[j].Vt = q.Vt;
      ta.lv[j].cheb = q.mem.cheb;
      ta.lv[j].m = q.m;
    }
    ta.b = c.b;
    ta.x = c.x;
    ta.done = done;
    ta.S = c.g.S;
    launch_mg_tail(ta, s);
  } else if (l + 2 < H.L) {
    mg_cycle(H, l + 1, s);
  }
  std::memset(&t, 0, sizeof(t));
  t.coarse_in = c.x;
  t.fine_x = v.x;
  t.done = done;
  t.op = MG_PROLONG;
  t.mc = c.m;
  t.S = c.g.S;
  t.Sp = c.g.Sp;
  launch_mg_transfer(t, s);
  std::memset(&a, 0, sizeof(a));
  a.V = v.V;
  a.m = v.mem;
  a.g = v.g;
  a.r = v.b;
  a.src = v.x;
  a.q = v.res;
  a.zout = v.za;
  a.cheb_init = 1;
  launch_fe3d<M_RESID>(a, s);
  std::memset(&a, 0, sizeof(a));
  a.V = v.V;
  a.m = v.mem;
  a.g = v.g;
  a.r = v.res;
  a.src = v.za;
  a.x = v.x;
  a.dotv = dotv;
  a.partial = partial;
  a.cheb_step = 1;
  launch_fe3d<M_CHEBX>(a, s);
}

// One V-cycle application z[1] = V(r) on level 0 (smoother started), the
// post-smoother's correction fused with the partial sums of r^T z, and the
// step's rho (and beta) from them.
static void mg_apply(const MgHierarchy& H, const Workspace& w, bool init, hipStream_t s) {
  const MgLevel& f = H.lv[0];
  mg_cycle(H, 0, s, f.b, w.partial);
  finish(w, f.g, f.g.groups, F_CHEB, s, 0.0, init ? 1 : 0);
}

struct SolveOut {
  int32_t* iters;
  int32_t* status;
  double* relres;
  int32_t* ens_iters;
  ens_stats* stats;
};

// Iterations between the host's checks of the done flag.  The loop keeps two
// intervals queued, so a solve runs on for up to two intervals of early-exit
// launches after it has finished; the flag copy and event of each check cost
// a few microseconds of device time.  Short solves of ensembles large enough
// that an interval of four iterations still outlasts its host-side launch
// work (about 2^19 member-rows and up) therefore start with short intervals,
// growing with the iteration count as sqrt(k) (the overrun then stays a
// small share of a solve of any length) to the fixed 16 of small ensembles
// and long solves.  On MI355X this made the 31^3, S = 32 solves 1 % (Jacobi)
// and 5 % (Chebyshev-4) faster and left the 512^2 workload unchanged; fixed
// short intervals cost small ensembles up to 9 % (512^2, S = 1).
static int poll_interval(const Opts& o, const Geometry& g, int it) {
  if (o.poll > 0) return o.poll;
  if (g.nelem < ((size_t)1 << 19)) return 16;
  int p = 4;
  while (p < 16 && (size_t)(2 * p) * (size_t)(2 * p) <= (size_t)it) p *= 2;
  return p;
}

// Host side of the done-flag polls: a pinned two-slot flag and two events,
// kept in a process-wide pool and reused by later solves on the same device
// (created only when every pooled one is in use, never freed), so a solve
// allocates nothing once the pool holds one per concurrent solve.
struct Poller {
  int dev;
  int32_t* flag;
  hipEvent_t ev[2];
};

static std::mutex g_poll_mu;
static std::vector<Poller*> g_poll_free;

static int acquire_poller(Poller** out) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_poll_mu);
    for (size_t k = 0; k < g_poll_free.size(); ++k) {
      if (g_poll_free[k]->dev == dev) {
        *out = g_poll_free[k];
        g_poll_free.erase(g_poll_free.begin() + (long)k);
        return ENS_OK;
      }
    }
  }
  Poller* p = new Poller;
  p->dev = dev;
  p->flag = nullptr;
  p->ev[0] = p->ev[1] = nullptr;
  hipError_t e = hipHostMalloc((void**)&p->flag, 2 * sizeof(int32_t), hipHostMallocDefault);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&p->ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    for (int k = 0; k < 2; ++k)
      if (p->ev[k]) (void)hipEventDestroy(p->ev[k]);
    if (p->flag) (void)hipHostFree(p->flag);
    delete p;
    return set_hip_error(e);
  }
  *out = p;
  return ENS_OK;
}

static void release_poller(Poller* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_poll_mu);
  g_poll_free.push_back(p);
}

// Clears the control words (a kernel rather than a memset node, so the
// clearing also behaves under stream capture).
__global__ void clear_ctl_kernel(int* ctl) {
  if (threadIdx.x < CTL_COUNT) ctl[threadIdx.x] = 0;
}

// How run_solve learns that every member has stopped.  POLL_ASYNC: copies
// of the done flag into pinned memory, checked one interval behind (two
// intervals stay queued).  POLL_SYNC: allocates nothing and creates no
// events: each check copies the flag to the host and waits for the stream
// (the queue drains once per interval).
enum PollMode { POLL_ASYNC = 0, POLL_SYNC = 1 };

static int run_solve(const ens_problem* prob, const Opts& o, int S, const double* V, const double* b,
                     int b_bcast, double* x, const Workspace& w, hipStream_t s, SolveOut out,
                     PollMode mode = POLL_ASYNC, const MgHierarchy* mgh = nullptr) {
  const bool mg = (o.precond == ENS_PRECOND_MULTIGRID);
  const bool cheb = uses_poly(o);   // Chebyshev or multigrid: smoother coefficients at init
  const Geometry g = geometry_for(prob, o, S);
  const int ge = init_groups(g);
  MgHierarchy H;
  if (mg) {
    if (!mgh || mgh->L < 2) return ENS_EINVAL;
    H = *mgh;
    H.levelwise = (o.flags & ENS_FLAG_MG_LEVELWISE) ? 1 : 0;
    mg_bind_fine(H, V, w, g);
    mg_setup(H, w, o.ratio, s);
  }

  hipLaunchKernelGGL(clear_ctl_kernel, dim3(1), dim3(64), 0, s, w.m.ctl);
  InitArgs ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.V = V;
  ia.b = b;
  ia.b_broadcast = b_bcast;
  ia.x = x;
  ia.p0 = w.p[0];
  ia.r = w.r;
  ia.partial = w.partial;
  ia.m = w.m;
  ia.g = g;
  ia.max_iter = o.max_iter;
  ia.cheb = cheb ? 1 : 0;
  ia.cheb_degree = o.degree;
  ia.cheb_ratio = o.ratio;
  launch_init(ia, ge, s);
  {
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = ge;
    f.kind = F_INIT;
    f.m = w.m;
    f.g = g;
    f.cheb = cheb ? 1 : 0;
    f.cheb_degree = o.degree;
    f.cheb_ratio = o.ratio;
    f.max_iter = o.max_iter;
    launch_finish(f, s);
  }
  double* zfinal = nullptr;
  if (mg) {
    launch_cheb_start(V, w.r, w.z[0], w.m, g, ge, s);
    mg_apply(H, w, true, s);
    zfinal = w.z[1];
  } else if (cheb) {
    zfinal = cheb_apply(V, w, g, o.degree, true, false, s);
  }
  HIPCHECK(hipGetLastError());

  const bool timing = (o.flags & ENS_FLAG_TIME_SPMV) != 0 && mode == POLL_ASYNC;
  std::vector<hipEvent_t> evs;
  std::vector<int> ev_iter;

  Poller* poller = nullptr;
  if (mode == POLL_ASYNC) {
    const int prc = acquire_poller(&poller);
    if (prc != ENS_OK) {
      (void)hipStreamSynchronize(s);
      return prc;
    }
  }
  int32_t* flag = poller ? poller->flag : nullptr;
  int rc = ENS_OK;
  auto fail = [&](hipError_t e) { rc = set_hip_error(e); };
  int it = 0, slot = 0;
  bool have_prev = false;
  while (rc == ENS_OK && it < o.max_iter) {
    const int chunk = std::min(poll_interval(o, g, it), o.max_iter - it);
    for (int c = 0; c < chunk; ++c) {
      ++it;
      StencilArgs a;
      std::memset(&a, 0, sizeof(a));
      a.V = V;
      a.r = w.r;
      a.src = zfinal;
      a.pold = w.p[(it + 1) & 1];
      a.pnew = w.p[it & 1];
      a.q = w.q;
      a.x = x;
      a.partial = w.partial;
      a.m = w.m;
      a.g = g;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timing && c == 0) {
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) { fail(e); break; }
        (void)hipEventRecord(e0, s);
      }
      if (cheb) launch_stencil<M_PCG_Z>(a, s);
      else launch_stencil<M_PCG_J>(a, s);
      if (e1) {
        (void)hipEventRecord(e1, s);
        evs.push_back(e0);
        evs.push_back(e1);
        ev_iter.push_back(it);
      }
      finish(w, g, g.groups, F_ALPHA, s);
      if (cheb && !mg && g.dim == 2) {
        // the residual update fused with the first Chebyshev step; the
        // residual alternates between two buffers (w.r holds the initial one)
        double* r_in = (it & 1) ? w.r : w.aux;
        double* r_out = (it & 1) ? w.aux : w.r;
        StencilArgs c;
        std::memset(&c, 0, sizeof(c));
        c.V = V;
        c.r = r_in;
        c.q_in = w.q;
        c.r_out = r_out;
        c.zout = w.z[1];
        c.partial = w.partial;
        c.m = w.m;
        c.g = g;
        c.cheb_step = 1;
        c.cheb_last = (o.degree == 2);
        launch_stencil<M_CHEB1>(c, s);
        finish(w, g, g.groups, F_UPDATE_C, s, o.rtol);
        cheb_apply(V, w, g, o.degree, false, true, s, r_out, 2);
      } else {
        UpdateArgs u;
        std::memset(&u, 0, sizeof(u));
        u.V = V;
        u.r = w.r;
        u.q = w.q;
        u.z = w.z[0];
        u.partial = w.partial;
        u.m = w.m;
        u.g = g;
        u.rtol = o.rtol;
        launch_update(u, cheb, ge, s);
        finish(w, g, ge, cheb ? F_UPDATE_C : F_UPDATE_J, s, o.rtol);
        if (mg) mg_apply(H, w, false, s);
        else if (cheb) cheb_apply(V, w, g, o.degree, false, true, s);
      }
    }
    if (rc != ENS_OK) break;
    hipError_t e = hipGetLastError();
    if (mode == POLL_SYNC) {
      int32_t done = 0;
      if (e == hipSuccess)
        e = hipMemcpyAsync(&done, w.m.ctl + CTL_DONE, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { fail(e); break; }
      if (done) break;
      continue;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag[slot], w.m.ctl + CTL_DONE, sizeof(int32_t),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(poller->ev[slot], s);
    if (e == hipSuccess && have_prev) e = hipEventSynchronize(poller->ev[slot ^ 1]);
    if (e != hipSuccess) { fail(e); break; }
    if (have_prev && flag[slot ^ 1]) break;
    have_prev = true;
    slot ^= 1;
  }
  if (rc == ENS_OK) launch_final(x, w.p[0], w.p[1], w.m, g, ge, s);

  int32_t h_iters[kMaxS], h_status[kMaxS];
  double h_relres[kMaxS];
  if (rc == ENS_OK) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h_iters, w.m.iters, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_status, w.m.status, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_relres, w.m.relres, sizeof(double) * S, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) fail(e);
  } else {
    (void)hipStreamSynchronize(s);
  }
  int ens_iters = 0;
  if (rc == ENS_OK) {
    for (int k = 0; k < S; ++k) ens_iters = std::max(ens_iters, (int)h_iters[k]);
    if (out.iters) std::memcpy(out.iters, h_iters, sizeof(int32_t) * S);
    if (out.status) std::memcpy(out.status, h_status, sizeof(int32_t) * S);
    if (out.relres) std::memcpy(out.relres, h_relres, sizeof(double) * S);
    if (out.ens_iters) *out.ens_iters = ens_iters;
  }
  if (out.stats) {
    ens_stats st;
    std::memset(&st, 0, sizeof(st));
    st.ens_iters = ens_iters;
    st.spmv_groups = g.groups;
    st.tile_lines = g.ty;
    for (size_t k = 0; k < ev_iter.size(); ++k) {
      if (rc == ENS_OK && ev_iter[k] <= ens_iters) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, evs[2 * k], evs[2 * k + 1]) == hipSuccess) {
          st.spmv_ms += ms;
          st.spmv_timed += 1;
        }
      }
    }
    *out.stats = st;
  }
  for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  release_poller(poller);   // the stream is idle: no copy into its flag is pending
  return rc;
}

// ------------------------------------------------------------ no-allocation solve
// Workspace of ens_pcg_solve_noalloc: a file-scope device array, one copy per
// device, held while the process lives.  Host code never uses the array's
// name as an address (on the host it names a stand-in, not device memory): the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address reaches kernels.
constexpr size_t kScratchBytes = (size_t)ENS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_for_current_device(void** out) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return ENS_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return ENS_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ENS_OK;
}

}  // namespace ens

using namespace ens;

extern "C" {

int ens_version(void) { return 100; }

int ens_stream_triad(const double* a_dev, const double* b_dev, double* c_dev, double scalar, size_t n,
                     void* stream) {
  if (!a_dev || !b_dev || !c_dev || n == 0 || !std::isfinite(scalar)) return ENS_EINVAL;
  const uintptr_t mis = ((uintptr_t)a_dev | (uintptr_t)b_dev | (uintptr_t)c_dev) & 15;
  if (mis) return ENS_EINVAL;
  launch_triad(a_dev, b_dev, c_dev, scalar, n, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  return ENS_OK;
}

int ens_stream_mix(const double* src_dev, double* dst_dev, size_t stride, size_t n, int32_t nread,
                   int32_t nwrite, void* stream) {
  if (!src_dev || !dst_dev || n < 2 || (n & 1) || stride < n || (stride & 1)) return ENS_EINVAL;
  if ((((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15) != 0) return ENS_EINVAL;
  const int rc = launch_stream_mix(src_dev, dst_dev, stride, n, nread, nwrite, (hipStream_t)stream);
  if (rc) return rc;
  HIPCHECK(hipGetLastError());
  return ENS_OK;
}

int ens_last_hip_error(void) { return g_last_hip_error; }

const char* ens_strerror(int code) {
  switch (code) {
    case ENS_OK: return "ok";
    case ENS_EINVAL: return "invalid argument";
    case ENS_ENOMEM: return "workspace too small";
    case ENS_EHIP: return "HIP runtime error";
    case ENS_ENOTSUP: return "unsupported";
    default: return "unknown error";
  }
}

// finite parameters only: the matrix of a member with a non-finite parameter
// would hold non-finite values
static int check_params(const double* y_host, int S, int d) {
  if (!y_host) return ENS_EINVAL;
  for (size_t k = 0; k < (size_t)S * d; ++k)
    if (!std::isfinite(y_host[k])) return ENS_EINVAL;
  return ENS_OK;
}

// members per assembly launch: as many as kAsmY parameter values hold
static int asm_chunk(int S, int d) { return std::max(1, std::min(S, kAsmY / d)); }

int ens_assemble_ensemble(const ens_problem* prob, int32_t S, const double* y_host, double* V_dev,
                          double* b_dev, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !b_dev) return ENS_EINVAL;
  rc = check_params(y_host, S, prob->d);
  if (rc) return rc;
  const int d = prob->d;
  const int mcmax = asm_chunk(S, d);
  hipStream_t st = (hipStream_t)stream;
  if (is3d(prob)) {
    Fe3dAsmArgs f;
    std::memset(&f, 0, sizeof(f));
    rc = fe3d_setup(prob, f);
    if (rc) return rc;
    f.V = V_dev;
    f.b = b_dev;
    f.m = prob->n;
    f.S = S;
    f.d = d;
    f.test = prob->eps_model;
    f.nr = rows_of(prob);
    f.vstride = slot_stride(f.nr * S);
    for (int m0 = 0; m0 < S; m0 += mcmax) {
      f.m0 = m0;
      f.mc = std::min(mcmax, S - m0);
      f.mcp = pow2ceil(f.mc);
      std::memcpy(f.y, y_host + (size_t)m0 * d, sizeof(double) * (size_t)f.mc * d);
      launch_fe3d_assemble(f, st);
    }
    HIPCHECK(hipGetLastError());
    return ENS_OK;
  }
  AsmArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = V_dev;
  a.b = b_dev;
  a.n = prob->n;
  a.S = S;
  a.d = d;
  a.eps_model = prob->eps_model;
  a.amp = prob->amp;
  a.ntx = (prob->n + kAsmTX - 1) / kAsmTX;
  a.vstride = slot_stride((size_t)prob->n * prob->n * S);
  for (int m0 = 0; m0 < S; m0 += mcmax) {
    a.m0 = m0;
    a.mc = std::min(mcmax, S - m0);
    a.mcp = pow2ceil(a.mc);
    std::memcpy(a.y, y_host + (size_t)m0 * d, sizeof(double) * (size_t)a.mc * d);
    launch_assemble(a, st);
  }
  HIPCHECK(hipGetLastError());
  return ENS_OK;
}

// The QoI weights (paper, Section 2.1: a spatial mean of u): 1 / count at the
// interior nodes inside [0.4, 0.6]^dim, 0 elsewhere, in row order.  A node
// index i (1-based) is inside when 2 (n + 1) <= 5 i <= 3 (n + 1), decided in
// integers.
__global__ void qoi_weights_kernel(double* w, int n, int dim, double inv_count, size_t nr) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  size_t rest = r;
  bool in = true;
  for (int q = 0; q < dim; ++q) {
    const long long i = (long long)(rest % (size_t)n) + 1;
    rest /= (size_t)n;
    in = in && 5 * i >= 2LL * (n + 1) && 5 * i <= 3LL * (n + 1);
  }
  w[r] = in ? inv_count : 0.0;
}

int ens_qoi_weights(const ens_problem* prob, double* w_dev, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!w_dev) return ENS_EINVAL;
  const int n = prob->n, dim = is3d(prob) ? 3 : 2;
  long long per = 0;
  for (long long i = 1; i <= n; ++i)
    if (5 * i >= 2LL * (n + 1) && 5 * i <= 3LL * (n + 1)) ++per;
  if (per == 0) return ENS_EINVAL;   // no node inside the box (n = 2)
  long long count = 1;
  for (int q = 0; q < dim; ++q) count *= per;
  const size_t nr = rows_of(prob);
  const unsigned blocks = (unsigned)((nr + kNT - 1) / kNT);
  hipLaunchKernelGGL(qoi_weights_kernel, dim3(blocks), dim3(kNT), 0, (hipStream_t)stream, w_dev, n,
                     dim, 1.0 / (double)count, nr);
  HIPCHECK(hipGetLastError());
  return ENS_OK;
}

size_t ens_matrix_slot_stride(const ens_problem* prob, int32_t S) {
  if (check_problem(prob) || !valid_S(S)) return 0;
  return slot_stride(rows_of(prob) * S);
}

size_t ens_pcg_workspace_bytes(const ens_problem* prob, const ens_opts* opts, int32_t S) {
  Opts o;
  if (check_problem(prob) || resolve_opts(opts, o) || !valid_S(S) || check_precond(prob, o)) return 0;
  return solve_bytes(prob, o, S);
}

int ens_pcg_solve(const ens_problem* prob, const ens_opts* opts, int32_t S, const double* V_dev,
                  const double* b_dev, double* x_dev, int32_t* iters_host, int32_t* status_host,
                  double* relres_host, int32_t* ens_iters_host, ens_stats* stats, void* ws_dev,
                  size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  Opts o;
  rc = resolve_opts(opts, o);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !b_dev || !x_dev || !ws_dev) return ENS_EINVAL;
  rc = check_precond(prob, o);
  if (rc) return rc;
  if (ws_bytes < solve_bytes(prob, o, S)) return ENS_ENOMEM;
  MgHierarchy H;
  const Workspace w = carve_solve(ws_dev, prob, o, S, &H);
  SolveOut out{iters_host, status_host, relres_host, ens_iters_host, stats};
  return run_solve(prob, o, S, V_dev, b_dev, 0, x_dev, w, (hipStream_t)stream, out, POLL_ASYNC, &H);
}

int ens_pcg_solve_noalloc(const ens_problem* prob, const ens_opts* opts, int32_t S,
                          const double* V_dev, const double* b_dev, double* x_dev,
                          int32_t* iters_host, int32_t* status_host, double* relres_host,
                          int32_t* ens_iters_host, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  Opts o;
  rc = resolve_opts(opts, o);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !b_dev || !x_dev) return ENS_EINVAL;
  rc = check_precond(prob, o);
  if (rc) return rc;
  if (solve_bytes(prob, o, S) > kScratchBytes) return ENS_ENOMEM;
  void* base = nullptr;
  rc = scratch_for_current_device(&base);
  if (rc) return rc;
  MgHierarchy H;
  const Workspace w = carve_solve(base, prob, o, S, &H);
  SolveOut out{iters_host, status_host, relres_host, ens_iters_host, nullptr};
  return run_solve(prob, o, S, V_dev, b_dev, 0, x_dev, w, (hipStream_t)stream, out, POLL_SYNC, &H);
}

int ens_spmv(const ens_problem* prob, int32_t S, const double* V_dev, const double* p_dev,
             double* q_dev, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !p_dev || !q_dev) return ENS_EINVAL;
  StencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = V_dev;
  a.src = p_dev;
  a.q = q_dev;
  if (is3d(prob)) {
    a.g = make_geometry3(prob->n, S);
  } else {
    a.g = make_geometry(prob->n, S, 0, 0);
    a.g.full = 1;   // any stored matrix, symmetric or not
  }
  launch_stencil<M_SPMV>(a, (hipStream_t)stream);
  HIPCHECK(hipGetLastError());
  return ENS_OK;
}

int ens_cheb_apply(const ens_problem* prob, const ens_opts* opts, int32_t S, const double* V_dev,
                   const double* r_dev, double* z_dev, double* lmax_host, void* ws_dev,
                   size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  Opts o;
  rc = resolve_opts(opts, o);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !r_dev || !z_dev || !ws_dev) return ENS_EINVAL;
  if (ws_bytes < workspace_bytes(rows_of(prob), S, true)) return ENS_ENOMEM;
  const Workspace w = carve_workspace(ws_dev, rows_of(prob), S, true);
  const Geometry g = geometry_for(prob, o, S);
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemsetAsync(w.m.ctl, 0, sizeof(int) * CTL_COUNT, s));
  InitArgs ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.V = V_dev;
  ia.b = r_dev;
  ia.x = w.aux;
  ia.p0 = w.p[0];
  ia.r = w.r;
  ia.partial = w.partial;
  ia.m = w.m;
  ia.g = g;
  ia.max_iter = 1;
  ia.cheb = 1;
  ia.cheb_degree = o.degree;
  ia.cheb_ratio = o.ratio;
  launch_init(ia, init_groups(g), s);
  {
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = init_groups(g);
    f.kind = F_INIT;
    f.m = w.m;
    f.g = g;
    f.cheb = 1;
    f.cheb_degree = o.degree;
    f.cheb_ratio = o.ratio;
    f.max_iter = 1;
    launch_finish(f, s);
  }
  // every member is preconditioned, whatever its residual: clear the done
  // flag the initialisation raises when all members have r = 0
  HIPCHECK(hipMemsetAsync(w.m.ctl + CTL_DONE, 0, sizeof(int), s));
  double* zf = cheb_apply(V_dev, w, g, o.degree, true, false, s);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(z_dev, zf, sizeof(double) * g.nelem, hipMemcpyDeviceToDevice, s));
  double lm[kMaxS];
  HIPCHECK(hipMemcpyAsync(lm, w.m.lmax, sizeof(double) * S, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (lmax_host) std::memcpy(lmax_host, lm, sizeof(double) * S);
  return ENS_OK;
}

int ens_mg_apply(const ens_problem* prob, const ens_opts* opts, int32_t S, const double* V_dev,
                 const double* r_dev, double* z_dev, double* lmax_host, void* ws_dev, size_t ws_bytes,
                 void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  ens_opts oo;
  if (opts) oo = *opts;
  else std::memset(&oo, 0, sizeof(oo));
  oo.precond = ENS_PRECOND_MULTIGRID;
  Opts o;
  rc = resolve_opts(&oo, o);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !r_dev || !z_dev || !ws_dev) return ENS_EINVAL;
  rc = check_precond(prob, o);
  if (rc) return rc;
  if (ws_bytes < solve_bytes(prob, o, S)) return ENS_ENOMEM;
  MgHierarchy H;
  const Workspace w = carve_solve(ws_dev, prob, o, S, &H);
  const Geometry g = geometry_for(prob, o, S);
  hipStream_t s = (hipStream_t)stream;
  H.levelwise = (o.flags & ENS_FLAG_MG_LEVELWISE) ? 1 : 0;
  mg_bind_fine(H, V_dev, w, g);
  mg_setup(H, w, o.ratio, s);
  hipLaunchKernelGGL(clear_ctl_kernel, dim3(1), dim3(64), 0, s, w.m.ctl);
  InitArgs ia;
  std::memset(&ia, 0, sizeof(ia));
  ia.V = V_dev;
  ia.b = r_dev;
  ia.x = w.p[1];
  ia.p0 = w.p[0];
  ia.r = w.r;
  ia.partial = w.partial;
  ia.m = w.m;
  ia.g = g;
  ia.max_iter = 1;
  ia.cheb = 1;
  ia.cheb_degree = kMgDegree;
  ia.cheb_ratio = o.ratio;
  launch_init(ia, init_groups(g), s);
  {
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = init_groups(g);
    f.kind = F_INIT;
    f.m = w.m;
    f.g = g;
    f.cheb = 1;
    f.cheb_degree = kMgDegree;
    f.cheb_ratio = o.ratio;
    f.max_iter = 1;
    launch_finish(f, s);
  }
  // every member is preconditioned, whatever its residual
  hipLaunchKernelGGL(clear_ctl_kernel, dim3(1), dim3(64), 0, s, w.m.ctl);
  launch_cheb_start(V_dev, w.r, w.z[0], w.m, g, init_groups(g), s);
  mg_apply(H, w, true, s);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(z_dev, w.z[1], sizeof(double) * g.nelem, hipMemcpyDeviceToDevice, s));
  double lm[kMaxS];
  HIPCHECK(hipMemcpyAsync(lm, w.m.lmax, sizeof(double) * S, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (lmax_host) std::memcpy(lmax_host, lm, sizeof(double) * S);
  return ENS_OK;
}

int ens_member_dot(int32_t N_r, int32_t S, const double* a_dev, const double* b_dev,
                   int32_t b_broadcast, double* out_host, void* ws_dev, size_t ws_bytes,
                   void* stream) {
  if (N_r < 1 || !valid_S(S) || !a_dev || !b_dev || !out_host || !ws_dev) return ENS_EINVAL;
  if (ws_bytes < header_bytes()) return ENS_ENOMEM;
  const Workspace w = carve_workspace(ws_dev, 0, S, false);
  Geometry g = make_geometry(2, S, 0, 0);
  g.nr = (size_t)N_r;
  g.nelem = (size_t)N_r * S;
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemsetAsync(w.m.ctl, 0, sizeof(int) * CTL_COUNT, s));
  launch_dot(a_dev, b_dev, b_broadcast ? 1 : 0, w.partial, g, init_groups(g), s);
  {
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = init_groups(g);
    f.kind = F_DOT;
    f.m = w.m;
    f.g = g;
    f.nsum = 1;
    f.scale = 1.0;
    launch_finish(f, s);
  }
  HIPCHECK(hipGetLastError());
  double res[kMaxS * 16];
  HIPCHECK(hipMemcpyAsync(res, w.m.result, sizeof(double) * S * 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int k = 0; k < S; ++k) out_host[k] = res[k * 16];
  return ENS_OK;
}

// 3-D model: grad_host[s][j] = -lambda_s^T (dA_s/dy_j) u_s (cube by cube)
static int dqdy3(const ens_problem* prob, int32_t S, const double* y_dev, const double* u_dev,
                 const double* lambda_dev, double* grad_host, void* ws_dev, void* stream) {
  const Workspace w = carve_workspace(ws_dev, 0, S, false);
  Geometry lanes;
  std::memset(&lanes, 0, sizeof(lanes));
  member_lanes(lanes, S);
  Fe3dDqdyArgs a;
  std::memset(&a, 0, sizeof(a));
  Fe3dAsmArgs f;
  std::memset(&f, 0, sizeof(f));
  int rc = fe3d_setup(prob, f);
  if (rc) return rc;
  std::memcpy(a.term, f.term, sizeof(a.term));
  a.y = y_dev;
  a.u = u_dev;
  a.lam = lambda_dev;
  a.partial = w.partial;
  a.m = prob->n;
  a.S = S;
  a.Sp = pow2ceil(S);
  a.d = prob->d;
  a.test = prob->eps_model;
  a.ncell = (size_t)(prob->n + 1) * (prob->n + 1) * (prob->n + 1);
  // d <= 16 partial arrays of groups * Sp doubles must fit the partial buffer
  const int groups = (int)std::min<size_t>((a.ncell * a.Sp + kNT - 1) / kNT,
                                           (size_t)(3 * kMaxGroups / kMaxTerms));
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemsetAsync(w.m.ctl, 0, sizeof(int) * CTL_COUNT, s));
  launch_fe3d_dqdy(a, groups, s);
  {
    FinishArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.partial = w.partial;
    fa.G = groups;
    fa.kind = F_SUMS;
    fa.m = w.m;
    fa.g = lanes;
    fa.g.vec = 1;        // one member per thread: slots Sp = pow2ceil(S)
    fa.g.tpp = fa.g.Sp = pow2ceil(S);
    fa.nsum = prob->d;
    fa.scale = -1.0;
    launch_finish(fa, s);
  }
  HIPCHECK(hipGetLastError());
  double res[kMaxS * 16];
  HIPCHECK(hipMemcpyAsync(res, w.m.result, sizeof(double) * S * 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < prob->d; ++j) grad_host[(size_t)k * prob->d + j] = res[k * 16 + j];
  return ENS_OK;
}

// copy the caller's parameters into the workspace (the blocking entry points
// synchronise the stream before returning, so the host array is read in time)
static int stage_params(const Workspace& w, const double* y_host, int S, int d, hipStream_t s) {
  HIPCHECK(hipMemcpyAsync(w.y, y_host, sizeof(double) * (size_t)S * d, hipMemcpyHostToDevice, s));
  return ENS_OK;
}

int ens_param_indicator(const ens_problem* prob, int32_t S, const double* y_host, double* h_host,
                        void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!valid_S(S) || !h_host || !ws_dev) return ENS_EINVAL;
  rc = check_params(y_host, S, prob->d);
  if (rc) return rc;
  if (ws_bytes < header_bytes()) return ENS_ENOMEM;
  const Workspace w = carve_workspace(ws_dev, 0, S, false);
  rc = stage_params(w, y_host, S, prob->d, (hipStream_t)stream);
  if (rc) return rc;
  IndArgs a;
  std::memset(&a, 0, sizeof(a));
  if (is3d(prob)) {
    Fe3dAsmArgs f;
    std::memset(&f, 0, sizeof(f));
    rc = fe3d_setup(prob, f);
    if (rc) return rc;
    std::memcpy(a.term, f.term, sizeof(a.term));
    a.dim = 3;
    a.ncell = (size_t)(prob->n + 1) * (prob->n + 1) * (prob->n + 1);
  } else {
    a.dim = 2;
    a.ncell = 1;
  }
  a.y = w.y;
  a.partial = w.partial;
  a.m = prob->n;
  a.S = S;
  a.Sp = pow2ceil(S);
  a.d = prob->d;
  a.eps_model = prob->eps_model;
  const int groups = (int)std::min<size_t>((a.ncell * a.Sp + kNT - 1) / kNT, 512);
  hipStream_t s = (hipStream_t)stream;
  launch_indicator(a, groups, s);
  {
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = groups;
    f.kind = F_MAX;
    f.m = w.m;
    member_lanes(f.g, S);
    f.g.vec = 1;         // one member per thread: slots Sp = pow2ceil(S)
    f.g.tpp = f.g.Sp = pow2ceil(S);
    launch_finish(f, s);
  }
  HIPCHECK(hipGetLastError());
  double res[kMaxS * 16];
  HIPCHECK(hipMemcpyAsync(res, w.m.result, sizeof(double) * S * 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int k = 0; k < S; ++k) h_host[k] = res[k * 16];
  return ENS_OK;
}

// dQ/dy kernel on parameters already in the workspace
static int dqdy_staged(const ens_problem* prob, int32_t S, const double* u_dev,
                       const double* lambda_dev, double* grad_host, void* ws_dev, void* stream) {
  const Workspace w = carve_workspace(ws_dev, 0, S, false);
  if (is3d(prob)) return dqdy3(prob, S, w.y, u_dev, lambda_dev, grad_host, ws_dev, stream);
  const Geometry g = make_geometry(prob->n, S, 0, 0);
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemsetAsync(w.m.ctl, 0, sizeof(int) * CTL_COUNT, s));
  DqdyArgs a;
  a.y = w.y;
  a.u = u_dev;
  a.lam = lambda_dev;
  a.partial = w.partial;
  a.g = g;
  a.d = prob->d;
  a.eps_model = prob->eps_model;
  a.amp = prob->amp;
  a.ntx = (prob->n + kAsmTX - 1) / kAsmTX;
  a.ntiles = a.ntx * ((prob->n + kAsmTY - 1) / kAsmTY);
  // the partial buffer holds 3 * kMaxGroups * kMaxS doubles: d arrays of
  // groups * Sp partials; at most kMaxGroups workgroups (one tile each when
  // the grid has that few)
  const int cap = (int)std::min<size_t>((size_t)3 * kMaxGroups * kMaxS / ((size_t)prob->d * g.Sp),
                                        (size_t)kMaxGroups);
  const int groups = std::min(a.ntiles, cap);
  launch_dqdy(a, groups, s);
  {
    // dQ/dy_j = -(n+1)^2 * (the face/node sums of h^2 lambda^T dA/dy_j u)
    FinishArgs f;
    std::memset(&f, 0, sizeof(f));
    f.partial = w.partial;
    f.G = groups;
    f.kind = F_SUMS;
    f.m = w.m;
    f.g = g;
    f.nsum = prob->d;
    f.scale = -(double)(prob->n + 1) * (double)(prob->n + 1);
    launch_finish(f, s);
  }
  HIPCHECK(hipGetLastError());
  double res[kMaxS * 16];
  HIPCHECK(hipMemcpyAsync(res, w.m.result, sizeof(double) * S * 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < prob->d; ++j) grad_host[(size_t)k * prob->d + j] = res[k * 16 + j];
  return ENS_OK;
}

int ens_dqdy(const ens_problem* prob, int32_t S, const double* y_host, const double* u_dev,
             const double* lambda_dev, double* grad_host, void* ws_dev, size_t ws_bytes,
             void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!valid_S(S) || !u_dev || !lambda_dev || !grad_host || !ws_dev) return ENS_EINVAL;
  rc = check_params(y_host, S, prob->d);
  if (rc) return rc;
  if (ws_bytes < header_bytes()) return ENS_ENOMEM;
  const Workspace w = carve_workspace(ws_dev, 0, S, false);
  rc = stage_params(w, y_host, S, prob->d, (hipStream_t)stream);
  if (rc) return rc;
  return dqdy_staged(prob, S, u_dev, lambda_dev, grad_host, ws_dev, stream);
}

int ens_adjoint_grad(const ens_problem* prob, const ens_opts* opts, int32_t S, const double* y_host,
                     const double* V_dev, const double* u_dev, const double* w_dev,
                     double* lambda_dev, double* grad_host, int32_t* iters_host,
                     int32_t* status_host, void* ws_dev, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  Opts o;
  rc = resolve_opts(opts, o);
  if (rc) return rc;
  if (!valid_S(S) || !V_dev || !u_dev || !w_dev || !lambda_dev || !grad_host || !ws_dev)
    return ENS_EINVAL;
  rc = check_params(y_host, S, prob->d);
  if (rc) return rc;
  rc = check_precond(prob, o);
  if (rc) return rc;
  if (ws_bytes < solve_bytes(prob, o, S)) return ENS_ENOMEM;
  MgHierarchy H;
  const Workspace w = carve_solve(ws_dev, prob, o, S, &H);
  SolveOut out{iters_host, status_host, nullptr, nullptr, nullptr};
  rc = run_solve(prob, o, S, V_dev, w_dev, 1, lambda_dev, w, (hipStream_t)stream, out, POLL_ASYNC, &H);
  if (rc) return rc;
  rc = stage_params(w, y_host, S, prob->d, (hipStream_t)stream);
  if (rc) return rc;
  return dqdy_staged(prob, S, u_dev, lambda_dev, grad_host, ws_dev, stream);
}

}  // extern "C"
