// C ABI of libasdg: problem handle, device-buffer planning, factorisation,
// coarse setup and the preconditioned CG driver (Sec. 7 protocol).
//
// Device memory is caller-owned (four buffers, sizes from asdg_plan). The
// CG loop runs entirely on the device: every kernel reads the iteration
// state (iteration count, done flag, CG scalars) from device memory, so a
// chunk of `check_every` iterations can be captured once as a hipGraph and
// replayed; the host reads the state back only between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <cstdio>
#include <map>
#include <mutex>
#include <vector>

#include "asdg.h"
#include "discretize.h"
#include "kernels.h"

using namespace asdg;

namespace {

// Device workspace of asdg_apply_operator_static (the one entry point that
// works without the caller's bound scratch buffer): the input and the
// output of the operator apply in the internal, subdomain-major DoF order.
// Host code never passes this name to a kernel; it uses the address that
// hipGetSymbolAddress returns for the current device (static_scratch()).
constexpr int64_t kStaticMaxDofs = 1572864;
static __device__ __align__(256) double scratch[2 * kStaticMaxDofs];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy at its own address).
hipError_t static_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct Layout {
  size_t size = 0;
  size_t add(size_t bytes) {
    size_t o = (size + 255) & ~(size_t)255;
    size = o + std::max<size_t>(bytes, 1);
    return o;
  }
};

// Extreme eigenvalues of the symmetric tridiagonal matrix (d, e) by Sturm
// bisection (count of eigenvalues below x from the LDL^T pivots).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double& lmin, double& lmax) {
  size_t k = d.size();
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < k; ++i) {
    double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto kth = [&](int target) {  // smallest x with count(x) >= target
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      double m = 0.5 * (a + b);
      if (sturm_count(d, e, m) >= target) b = m; else a = m;
      if (b - a <= 1e-15 * std::max(std::fabs(a), std::fabs(b))) break;
    }
    return 0.5 * (a + b);
  };
  lmin = kth(1);
  lmax = kth((int)k);
}

// Copy of a caller mesh (the fine mesh is needed again by asdg_plan).
struct TetCopy {
  std::vector<double> xyz;
  std::vector<int32_t> tets;
  void assign(const asdg_tet_mesh& m) {
    xyz.assign(m.xyz, m.xyz + 3 * (size_t)m.n_vertices);
    tets.assign(m.tets, m.tets + 4 * (size_t)m.n_cells);
  }
  TetView view() const { return TetView{(int32_t)(xyz.size() / 3), xyz.data(), (int32_t)(tets.size() / 4), tets.data()}; }
};

struct MeshCopy {
  std::vector<double> xy;
  std::vector<int32_t> ptr, verts;
  void assign(const asdg_mesh& m) {
    xy.assign(m.xy, m.xy + 2 * (size_t)m.n_vertices);
    ptr.assign(m.cell_ptr, m.cell_ptr + m.n_cells + 1);
    verts.assign(m.cell_vertices, m.cell_vertices + m.cell_ptr[m.n_cells]);
  }
  MeshView view() const {
    return MeshView{(int32_t)(xy.size() / 2), xy.data(), (int32_t)ptr.size() - 1, ptr.data(), verts.data()};
  }
};

}  // namespace

struct asdg_problem {
  std::string err;
  MeshCopy fine;
  TetCopy tet;  // 3D fine mesh (A.dim == 3)
  int stage = 0;  // 1 assembled, 2 planned, 3 bound, 4 factored
  bool coarse_ready = false;
  Assembled A;
  Coarse C;
  bool has_coarse = false;
  int f32 = 0;
  int32_t n0 = 0;
  std::vector<double> rhs_caller;
  // local factor planning
  int tile = TILE;        // tile edge of the local factors (64 or 32; the coarse factor always TILE)
  int tile_req = 0;       // ASDG_TUNE_TILE: 0 automatic (64, the autotuner may switch), 32 or 64 fixed
  bool tile_search = false;  // buffers planned for both edges (the autotuner may switch the layout)
  std::vector<SubDesc> subs;
  std::vector<int4> tile_meta, chol_tasks, trsv_tasks;
  int64_t n_tiles = 0;
  int32_t max_n = 0;
  // coarse factor planning
  SubDesc csub{0, 0, 0, 0};
  std::vector<int4> cchol_tasks, ctrsv_tasks;
  std::vector<double, DefaultInit<double>> ctiles_host;  // every element written by plan_coarse_factor
  int64_t n_ctiles = 0;
  // buffer layout
  struct { size_t row_ptr, col, blocks, rhs, perm, cell_sub; } o0{};
  struct { size_t tiles, subs, chol, trsv, meta, xtiles, inv, subt, colt; } o1{};
  struct { size_t pptr, pcol, pval, tptr, tcell, tblk, ctiles, csub, cchol, ctrsv, cS, cX, cinv, cmeta, cinvt; } o2{};
  // coarse solve by a dense explicit A_0^{-1} (n0 <= kCoarseDenseMax) instead of the triangular sweeps
  bool coarse_dense = false;
  // with the explicit inverse: applied from its packed lower tiles (half the
  // bytes, three small launches) instead of the expanded dense matrix
  bool coarse_packed = false;
  int coarse_packed_mode = 0;  // 0: packed from kCoarsePackedMin on, 1: always packed, 2: always dense
  int rsplits = 1;  // work-groups per coarse cell in the restriction (partials added by the dense coarse solve)
  std::vector<int4> cmeta, cinv_tasks;
  struct { size_t x, r, p, q, z, yl, zl, r0, y0, z0, red, st, rz2, ah, bh, flags, trace, part, cpart; } o3{};
  size_t bytes[4] = {0, 0, 0, 0};
  char* buf[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t failed_sub = -2;
  int n_cu = 256;
  int chol_per_cu = 0, trsv_per_cu = 0, chol_grid = 0, trace = 0;  // 0: defaults
  int inv_per_cu = 0, symv_waves = 0;                                // 0: defaults
  int task_chunk = 0;        // subdomains per group of the factorisation task order (0: all at once)
  // factorisation schedule: 0 automatic, 1 tile tasks (Cholesky and X = L^{-1}), 2 one work-group per
  // subdomain (Cholesky) and per block column (X = L^{-1})
  int factor_sched = 0, inv_sched = 0;
  std::vector<int4> sub_tasks, col_tasks;  // the schedule-2 queues, largest work first
  int host_threads = 0;      // cap on host threads of assembly and planning (0: default)
  std::string arch;          // device architecture name (set by asdg_bind)
  bool tasks_dirty = false;  // task lists reordered after asdg_bind, not yet uploaded
  int local_inverse = 0, inv_planned = 0;  // explicit local inverses (set before asdg_plan)
  // small-subdomain mode: every n_i <= TILE; A_i^{-1} stored whole (n_i^2 words at subs[i].tile0) and
  // applied inside the prolongation; no tiles, no local launch
  int small_off = 0;
  int no_precond = 0;  // identity preconditioner (plain CG; Lanczos then estimates K(A))
  bool small = false;
  int64_t small_words = 0;
  std::vector<int4> inv_tasks;
  std::vector<int32_t> cell_sub;
  // captured iteration chunk
  hipGraphExec_t gexec = nullptr;
  int g_k = 0, g_timed = 0;
  hipStream_t own_stream = nullptr;
  // the coarse correction (restriction + dense coarse solve) runs on side_stream
  // beside the local solves; fork/join through events (graph edges when captured)
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  std::vector<hipEvent_t> ev;  // 2 per captured iteration (local solve start/end)
  hipEvent_t t0 = nullptr, t1 = nullptr;
  // non-blocking solve state
  DevState* h_state = nullptr;  // pinned host copy target
  hipEvent_t chunk_ev = nullptr;
  bool chunk_in_flight = false, solve_open = false;
  DevState hs{};
  asdg_pcg_opts aopts{1e-8, 20000, 16, 1, 0};
  const double* solve_b = nullptr;  // right-hand side of the open solve (caller order), for the true residual
  // host wall times of the setup phases (reported in asdg_pcg_stats)
  double t_assemble_ms = 0.0, t_coarse_host_ms = 0.0, t_factor_ms = 0.0, t_coarse_dev_ms = 0.0;

  template <class T>
  T* ptr(int b, size_t off) const { return reinterpret_cast<T*>(buf[b] + off); }
  int64_t n() const { return (int64_t)A.n_cells * A.np; }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    g_k = 0;
  }
  ~asdg_problem() {
    drop_graph();
    for (auto e : ev) (void)hipEventDestroy(e);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (chunk_ev) (void)hipEventDestroy(chunk_ev);
    if (h_state) (void)hipHostFree(h_state);
  }
};

static double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Records the wall time of the enclosing scope into `out` (every return path).
struct WallTimer {
  double& out;
  double t0;
  explicit WallTimer(double& o) : out(o), t0(wall_ms()) {}
  ~WallTimer() { out = wall_ms() - t0; }
};

#define FAIL(pb, code, msg) \
  do {                      \
    (pb)->err = (msg);      \
    return (code);          \
  } while (0)
#define HIPCHK(pb, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) FAIL(pb, ASDG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

asdg_status asdg_create(asdg_problem** out) {
  if (!out) return ASDG_EINVAL;
  *out = new (std::nothrow) asdg_problem();
  return *out ? ASDG_OK : ASDG_ENOMEM;
}

void asdg_destroy(asdg_problem* pb) { delete pb; }

const char* asdg_last_error(const asdg_problem* pb) { return pb ? pb->err.c_str() : "null handle"; }

asdg_status asdg_assemble(asdg_problem* pb, const asdg_mesh* fine, int32_t p, double c_sigma, const double* rho,
                          const int32_t* subdomain, asdg_field_fn f, void* f_user) {
  if (!pb) return ASDG_EINVAL;
  if (!fine || !fine->xy || !fine->cell_ptr || !fine->cell_vertices || !rho || !subdomain || fine->n_cells < 1)
    FAIL(pb, ASDG_EINVAL, "null or empty input");
  pb->drop_graph();
  pb->stage = 0;
  pb->coarse_ready = false;
  MeshView mv{fine->n_vertices, fine->xy, fine->n_cells, fine->cell_ptr, fine->cell_vertices};
  HostThreadCap cap(pb->host_threads);
  const double ta = wall_ms();
  std::string e = assemble_sipg(mv, p, c_sigma, rho, subdomain, f, f_user, pb->A);
  pb->t_assemble_ms = wall_ms() - ta;
  if (!e.empty()) FAIL(pb, ASDG_EINVAL, e);
  const int np = pb->A.np;
  pb->rhs_caller.assign(pb->A.rhs.size(), 0.0);
  for (int32_t r = 0; r < pb->A.n_cells; ++r)
    for (int a = 0; a < np; ++a) pb->rhs_caller[(size_t)pb->A.perm[r] * np + a] = pb->A.rhs[(size_t)r * np + a];
  pb->fine.assign(*fine);  // kept for the coarse transfer
  pb->tet = TetCopy();
  pb->stage = 1;
  return ASDG_OK;
}

asdg_status asdg_assemble_tet(asdg_problem* pb, const asdg_tet_mesh* fine, int32_t p, double c_sigma,
                              const double* rho, const int32_t* subdomain, asdg_field_fn f, void* f_user) {
  if (!pb) return ASDG_EINVAL;
  if (!fine || !fine->xyz || !fine->tets || !rho || !subdomain || fine->n_cells < 1 || fine->n_vertices < 4)
    FAIL(pb, ASDG_EINVAL, "null or empty input");
  pb->drop_graph();
  pb->stage = 0;
  pb->coarse_ready = false;
  TetView tv{fine->n_vertices, fine->xyz, fine->n_cells, fine->tets};
  HostThreadCap cap(pb->host_threads);
  const double ta = wall_ms();
  std::string e = assemble_sipg_tet(tv, p, c_sigma, rho, subdomain, f, f_user, pb->A);
  pb->t_assemble_ms = wall_ms() - ta;
  if (!e.empty()) FAIL(pb, ASDG_EINVAL, e);
  const int np = pb->A.np;
  pb->rhs_caller.assign(pb->A.rhs.size(), 0.0);
  for (int32_t r = 0; r < pb->A.n_cells; ++r)
    for (int a = 0; a < np; ++a) pb->rhs_caller[(size_t)pb->A.perm[r] * np + a] = pb->A.rhs[(size_t)r * np + a];
  pb->tet.assign(*fine);  // kept for the coarse transfer
  pb->fine = MeshCopy();
  pb->stage = 1;
  return ASDG_OK;
}

}  // extern "C"

namespace {

// Longest path (in units of one 64x64x64 tile product) from each task
// (j, b) of a tile Cholesky with nb block columns to the end of the
// factorisation: task (j, b) runs j updates, then the diagonal factor and
// inverse (about ten units) or one product with inv(L_jj); its consumers
// are (j', b) for j < j' <= b and (b, b') for b' >= b, and the diagonal
// task feeds (j, b') for b' > j. Entry [j * nb + b].
static std::vector<int32_t> cholesky_levels(int nb) {
  std::vector<int32_t> lv((size_t)nb * nb, 0);
  for (int j = nb - 1; j >= 0; --j)
    for (int b = nb - 1; b >= j; --b) {
      int32_t m = 0;
      if (b == j) {
        for (int b2 = j + 1; b2 < nb; ++b2) m = std::max(m, lv[j * nb + b2]);
      } else {
        for (int j2 = j + 1; j2 <= b; ++j2) m = std::max(m, lv[j2 * nb + b]);
        for (int b2 = b; b2 < nb; ++b2) m = std::max(m, lv[b * nb + b2]);
      }
      lv[j * nb + b] = m + j + (b == j ? 10 : 1);
    }
  return lv;
}

// The same for X = L^{-1}: task (j, b) runs b - j updates and one product
// with D_b (a copy when b == j); its consumers are (j, b') for b' > b.
static std::vector<int32_t> inverse_levels(int nb) {
  std::vector<int32_t> lv((size_t)nb * nb, 0);
  for (int j = 0; j < nb; ++j)
    for (int b = nb - 1; b >= j; --b) {
      int32_t m = 0;
      for (int b2 = b + 1; b2 < nb; ++b2) m = std::max(m, lv[j * nb + b2]);
      lv[j * nb + b] = m + (b - j) + 1;
    }
  return lv;
}

// Tasks (i, j, b), j <= b < nb_i, of every subdomain, longest path first
// (ties by subdomain, column, row); every dependency has a strictly longer
// path, so it precedes its consumers. chunk > 0: subdomains in groups of
// chunk consecutive ones, group by group (a smaller working set at a time).
static std::vector<int4> order_tasks(const std::vector<SubDesc>& subs, std::vector<int32_t> (*levels)(int),
                                     int chunk) {
  struct K { int32_t g, lv, i, j, b; };
  std::vector<K> ks;
  std::map<int, std::vector<int32_t>> memo;
  for (int32_t i = 0; i < (int32_t)subs.size(); ++i) {
    const int nb = subs[i].nb;
    auto it = memo.find(nb);
    if (it == memo.end()) it = memo.emplace(nb, levels(nb)).first;
    for (int j = 0; j < nb; ++j)
      for (int b = j; b < nb; ++b) ks.push_back({chunk > 0 ? i / chunk : 0, it->second[(size_t)j * nb + b], i, j, b});
  }
  std::sort(ks.begin(), ks.end(), [](const K& x, const K& y) {
    if (x.g != y.g) return x.g < y.g;
    if (x.lv != y.lv) return x.lv > y.lv;
    if (x.i != y.i) return x.i < y.i;
    if (x.j != y.j) return x.j < y.j;
    return x.b < y.b;
  });
  std::vector<int4> out(ks.size());
  for (size_t k = 0; k < ks.size(); ++k) out[k] = make_int4(ks[k].i, ks[k].j, ks[k].b, 0);
  return out;
}

// Block-column tasks (i, j) of X = L^{-1} (schedule 2), largest work first
// (the column's tile products, about (nb - j)^2 / 2; ties by subdomain,
// column). chunk > 0: subdomains in groups of chunk consecutive ones, group
// by group, so the columns running together share their subdomain's L tiles
// in the caches.
static std::vector<int4> order_col_tasks(const std::vector<SubDesc>& subs, int chunk) {
  struct C { int32_t g; int64_t w; int32_t i, j; };
  std::vector<C> cs;
  for (int32_t i = 0; i < (int32_t)subs.size(); ++i) {
    const int64_t nb = subs[i].nb;
    for (int j = 0; j < nb; ++j) cs.push_back({chunk > 0 ? i / chunk : 0, (nb - j) * (nb - j + 1) / 2, i, j});
  }
  std::stable_sort(cs.begin(), cs.end(), [](const C& a, const C& b) { return a.g != b.g ? a.g < b.g : a.w > b.w; });
  std::vector<int4> out(cs.size());
  for (size_t k = 0; k < cs.size(); ++k) out[k] = make_int4(cs[k].i, cs[k].j, 0, 0);
  return out;
}

// Stored tiles and sweep tasks of the local tile layout with edge t.
void local_counts(const asdg_problem* pb, int t, int64_t& tiles, int64_t& sweeps) {
  tiles = 0;
  sweeps = 0;
  for (int32_t i = 0; i < pb->A.n_sub; ++i) {
    const int64_t n = (int64_t)(pb->A.sub_ptr[i + 1] - pb->A.sub_ptr[i]) * pb->A.np;
    const int64_t nb = (n + t - 1) / t;
    tiles += nb * (nb + 1) / 2;
    sweeps += 2 * nb;
  }
}

void plan_local(asdg_problem* pb) {
  const Assembled& A = pb->A;
  const int np = A.np;
  const int32_t ns = A.n_sub;
  pb->subs.resize(ns);
  int64_t tiles = 0;
  int nbmax = 0;
  pb->max_n = 0;
  for (int32_t i = 0; i < ns; ++i) {
    SubDesc& s = pb->subs[i];
    s.dof0 = A.sub_ptr[i] * np;
    s.n = (A.sub_ptr[i + 1] - A.sub_ptr[i]) * np;
    s.nb = (s.n + pb->tile - 1) / pb->tile;
    s.tile0 = (int32_t)tiles;
    tiles += (int64_t)s.nb * (s.nb + 1) / 2;
    nbmax = std::max(nbmax, s.nb);
    pb->max_n = std::max(pb->max_n, s.n);
  }
  int64_t words = 0;
  for (const SubDesc& d : pb->subs) words += (int64_t)d.n * d.n;
  pb->small = !pb->small_off && pb->max_n <= TILE && words < 0x7fffffff;
  pb->tile_meta.clear();
  pb->chol_tasks.clear();
  pb->trsv_tasks.clear();
  if (pb->small) {
    int64_t off = 0;
    for (SubDesc& d : pb->subs) {
      d.tile0 = (int32_t)off;  // word offset of the whole inverse
      off += (int64_t)d.n * d.n;
    }
    pb->small_words = words;
    pb->n_tiles = 0;
    return;
  }
  pb->small_words = 0;
  pb->n_tiles = tiles;
  pb->tile_meta.reserve(tiles);
  for (int32_t i = 0; i < ns; ++i)
    for (int b = 0; b < pb->subs[i].nb; ++b)
      for (int j = 0; j <= b; ++j)  // w: rows of tile row b inside the subdomain
        pb->tile_meta.push_back(make_int4(i, b, j, std::min(pb->tile, pb->subs[i].n - pb->tile * b)));
  // factorisation tasks (i, j, b): longest path to the end first (ties by
  // subdomain, column, row); every dependency has a strictly longer path, so
  // it precedes its consumers in the queue
  pb->chol_tasks = order_tasks(pb->subs, cholesky_levels, pb->task_chunk);
  // schedule 2: whole subdomains (Cholesky), largest first (ties by index),
  // and block columns (X = L^{-1})
  {
    std::vector<int32_t> ord(ns);
    for (int32_t i = 0; i < ns; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return pb->subs[a].nb > pb->subs[b].nb; });
    pb->sub_tasks.resize(ns);
    for (int32_t k = 0; k < ns; ++k) pb->sub_tasks[k] = make_int4(ord[k], 0, 0, 0);
    pb->col_tasks = order_col_tasks(pb->subs, pb->task_chunk);
  }
  struct K { int64_t key; int4 t; };
  std::vector<K> ks;
  // sweep tasks: forward b at step b, backward b at step 2nb-1-b; all
  // subdomains start together, tasks of one step are contiguous in the queue
  ks.clear();
  for (int32_t i = 0; i < ns; ++i) {
    int nb = pb->subs[i].nb;
    int64_t off = 0;
    for (int b = 0; b < nb; ++b) {
      ks.push_back({((off + b) * ns + i), make_int4(i, 0, b, 0)});
      ks.push_back({((off + 2 * nb - 1 - b) * ns + i), make_int4(i, 1, b, 0)});
    }
  }
  std::stable_sort(ks.begin(), ks.end(), [](const K& a, const K& b) { return a.key < b.key; });
  pb->trsv_tasks.resize(ks.size());
  for (size_t k = 0; k < ks.size(); ++k) pb->trsv_tasks[k] = ks[k].t;
}

// Largest coarse dimension solved with a dense explicit inverse (8 n0^2
// bytes: 512 MiB at the limit). One dense product reads the same bytes as
// the two triangular sweeps over the packed factor, without their chain of
// dependent tile rows.
constexpr int32_t kCoarseDenseMax = 8192;
constexpr int32_t kCoarsePackedMin = 4096;  // below, one dense product beats the packed pass and its two extra launches

void plan_coarse_factor(asdg_problem* pb) {
  const int32_t n0 = pb->n0;
  const int nb = (n0 + TILE - 1) / TILE;
  pb->csub = SubDesc{0, n0, nb, 0};
  pb->n_ctiles = (int64_t)nb * (nb + 1) / 2;
  pb->ctiles_host.clear();
  pb->ctiles_host.resize((size_t)pb->n_ctiles * TILE * TILE);
  // packed lower tiles of A_0 (identity padding), one tile row per item
  std::vector<int2> tile_bj(pb->n_ctiles);
  for (int b = 0; b < nb; ++b)
    for (int j = 0; j <= b; ++j) tile_bj[b * (b + 1) / 2 + j] = make_int2(b, j);
  parallel_for(pb->n_ctiles * TILE, [&](int64_t lo, int64_t hi) {
    for (int64_t it = lo; it < hi; ++it) {
      const int64_t t = it / TILE;
      const int r = (int)(it - t * TILE), b = tile_bj[t].x, j = tile_bj[t].y;
      double* T = &pb->ctiles_host[(size_t)t * TILE * TILE + (size_t)r * TILE];
      const int gr = b * TILE + r;
      for (int c = 0; c < TILE; ++c) {
        const int gc = j * TILE + c;
        T[c] = (gr < n0 && gc < n0) ? pb->C.a0[(size_t)gr * n0 + gc] : (gr == gc ? 1.0 : 0.0);
      }
    }
  });
  pb->cchol_tasks.clear();
  for (int j = 0; j < nb; ++j)
    for (int b = j; b < nb; ++b) pb->cchol_tasks.push_back(make_int4(0, j, b, 0));
  pb->ctrsv_tasks.clear();
  for (int b = 0; b < nb; ++b) pb->ctrsv_tasks.push_back(make_int4(0, 0, b, 0));
  for (int b = nb - 1; b >= 0; --b) pb->ctrsv_tasks.push_back(make_int4(0, 1, b, 0));
  pb->coarse_dense = n0 <= kCoarseDenseMax;
  pb->coarse_packed = pb->coarse_dense && (pb->coarse_packed_mode == 1 ||
                                           (pb->coarse_packed_mode == 0 && n0 >= kCoarsePackedMin));
  // restriction: about 512 (entry, row) pairs per work-group, at most 32 work-groups per coarse cell
  if (pb->coarse_dense) {
    const int64_t pairs = (int64_t)pb->C.tptr.back() * pb->A.np;
    const int64_t per_cell = (pairs + pb->C.n_coarse - 1) / pb->C.n_coarse;
    pb->rsplits = (int)std::max<int64_t>(1, std::min<int64_t>(32, (per_cell + 511) / 512));
  } else {
    pb->rsplits = 1;
  }
  pb->cmeta.clear();
  pb->cinv_tasks.clear();
  if (pb->coarse_dense) {
    for (int b = 0; b < nb; ++b)
      for (int j = 0; j <= b; ++j) {
        pb->cmeta.push_back(make_int4(0, b, j, std::min(TILE, n0 - TILE * b)));
        pb->cinv_tasks.push_back(make_int4(0, j, b, 0));  // row order: X_kj (k < b) precede X_bj
      }
  }
}

// z0 = A_0^{-1} r0: dense explicit inverse, or the two triangular sweeps.
asdg_status enqueue_coarse_solve(asdg_problem* pb, const DevState* st_done, hipStream_t s) {
  if (pb->coarse_packed) {
    // r0 (sum of the restriction splits) into y0, the packed symmetric
    // product by tiles, then the per-entry sums of the tile partials
    const double* r0 = pb->ptr<double>(3, pb->o3.r0);
    if (pb->rsplits > 1) {
      HIPCHK(pb, launch_sum_splits(pb->n0, pb->rsplits, r0, pb->ptr<double>(3, pb->o3.y0), st_done, s));
      r0 = pb->ptr<double>(3, pb->o3.y0);
    }
    HIPCHK(pb, launch_symv_tiles(0, 4, (int32_t)pb->n_ctiles, pb->ptr<int4>(2, pb->o2.cmeta),
                                 pb->ptr<SubDesc>(2, pb->o2.csub), pb->ptr<void>(2, pb->o2.cS), r0,
                                 pb->ptr<void>(3, pb->o3.cpart), st_done, s));
    HIPCHK(pb, launch_tile_partials_sum(pb->n0, (pb->n0 + TILE - 1) / TILE, pb->ptr<double>(3, pb->o3.cpart),
                                        pb->ptr<double>(3, pb->o3.z0), st_done, s));
    return ASDG_OK;
  }
  if (pb->coarse_dense) {
    HIPCHK(pb, launch_dense_mv(pb->n0, pb->rsplits, pb->ptr<double>(2, pb->o2.cinv), pb->ptr<double>(3, pb->o3.r0),
                               pb->ptr<double>(3, pb->o3.z0), st_done, s));
    return ASDG_OK;
  }
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  const int cgrid = (int)std::min<int64_t>((int64_t)pb->ctrsv_tasks.size(), (int64_t)pb->n_cu);
  HIPCHK(pb, launch_trsv(0, TILE, (int32_t)pb->ctrsv_tasks.size(), pb->ptr<int4>(2, pb->o2.ctrsv),
                         pb->ptr<SubDesc>(2, pb->o2.csub), pb->ptr<void>(2, pb->o2.ctiles),
                         pb->ptr<double>(3, pb->o3.r0), pb->ptr<void>(3, pb->o3.y0), pb->ptr<void>(3, pb->o3.z0), st,
                         &st->q_coarse, cgrid, nullptr, s));
  return ASDG_OK;
}

LocalParts local_parts(asdg_problem* pb) {
  return LocalParts{pb->ptr<int32_t>(0, pb->o0.cell_sub), pb->ptr<SubDesc>(1, pb->o1.subs),
                    pb->small ? pb->ptr<void>(1, pb->o1.tiles) : pb->ptr<void>(3, pb->o3.part), pb->small ? 1 : 0};
}

// z = P^{-1} r and partials of r.z. iteration: the prolongation also takes
// the PCG stopping decision (see launch_prolong).
// The batched local solves of a tile path (packed inverses or triangular
// sweeps) on r; st_done (may be NULL) lets the packed apply skip its work
// once the solve has stopped.
asdg_status enqueue_local(asdg_problem* pb, hipStream_t s, const DevState* st_done) {
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  const double* r = pb->ptr<double>(3, pb->o3.r);
  if (pb->inv_planned) {
    const int waves = pb->symv_waves > 0 ? pb->symv_waves : 4;
    HIPCHK(pb, launch_symv_tiles(pb->f32, waves, (int32_t)pb->n_tiles, pb->ptr<int4>(1, pb->o1.meta),
                                 pb->ptr<SubDesc>(1, pb->o1.subs), pb->ptr<void>(1, pb->o1.tiles), r,
                                 pb->ptr<void>(3, pb->o3.part), st_done, s));
  } else {
    const int lgrid = (int)std::min<int64_t>((int64_t)pb->trsv_tasks.size(),
                                             (int64_t)pb->n_cu * (pb->trsv_per_cu > 0 ? pb->trsv_per_cu : 2));
    HIPCHK(pb, launch_trsv(pb->f32, pb->tile, (int32_t)pb->trsv_tasks.size(), pb->ptr<int4>(1, pb->o1.trsv),
                           pb->ptr<SubDesc>(1, pb->o1.subs), pb->ptr<void>(1, pb->o1.tiles), r,
                           pb->ptr<void>(3, pb->o3.yl), pb->ptr<void>(3, pb->o3.zl), st, &st->q_local, lgrid,
                           pb->trace ? pb->ptr<uint64_t>(3, pb->o3.trace) : nullptr, s));
  }
  return ASDG_OK;
}

asdg_status enqueue_precond(asdg_problem* pb, hipStream_t s, DevState* st_done, Reduction* red, bool iteration,
                            hipEvent_t ev0, hipEvent_t ev1) {
  const int np = pb->A.np;
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  const double* r = pb->ptr<double>(3, pb->o3.r);
  if (pb->no_precond) {
    const LocalParts id{nullptr, nullptr, nullptr, 2};
    if (ev0) HIPCHK(pb, hipEventRecord(ev0, s));
    if (ev1) HIPCHK(pb, hipEventRecord(ev1, s));
    HIPCHK(pb, launch_prolong(np, 3, pb->A.n_cells, nullptr, nullptr, nullptr, nullptr, nullptr, &id, pb->f32, r,
                              pb->ptr<double>(3, pb->o3.z), red, st_done, iteration ? spmv_parts(pb->n()) : 0,
                              iteration ? vec_parts(pb->n()) : 0, s));
    return ASDG_OK;
  }
  // with the dense coarse solve, the coarse correction runs beside the local
  // solves on the side stream. Small subdomains of at least 10 DoFs get a
  // launch of their own for that, into q, which is free between the
  // residual update and the next operator apply; below that the extra
  // launch and pass over q cost more than the overlap gains (measured), and
  // their solves stay inside the prolongation.
  const bool side = pb->has_coarse && pb->coarse_dense && pb->side_stream && (!pb->small || pb->max_n >= 10);
  const hipStream_t sc = side ? pb->side_stream : s;
  if (side) {
    HIPCHK(pb, hipEventRecord(pb->fork_ev, s));
    HIPCHK(pb, hipStreamWaitEvent(sc, pb->fork_ev, 0));
  }
  if (pb->has_coarse) {
    HIPCHK(pb, launch_restrict(np, pb->C.nq, pb->C.n_coarse, pb->rsplits, pb->ptr<int32_t>(2, pb->o2.tptr),
                               pb->ptr<int32_t>(2, pb->o2.tcell), pb->ptr<int32_t>(2, pb->o2.tblk),
                               pb->ptr<double>(2, pb->o2.pval), r, pb->ptr<double>(3, pb->o3.r0),
                               pb->coarse_dense ? nullptr : pb->ptr<double>(3, pb->o3.y0),
                               pb->coarse_dense ? nullptr : pb->ptr<double>(3, pb->o3.z0), st_done, sc));
  }
  if (side) {
    asdg_status ce = enqueue_coarse_solve(pb, st_done, sc);
    if (ce != ASDG_OK) return ce;
    HIPCHK(pb, hipEventRecord(pb->join_ev, sc));
  }
  if (ev0) HIPCHK(pb, hipEventRecord(ev0, s));
  double* zloc = pb->ptr<double>(3, pb->o3.q);
  if (!pb->small) {
    asdg_status le = enqueue_local(pb, s, st);
    if (le != ASDG_OK) return le;
  } else if (side) {
    const LocalParts lp = local_parts(pb);
    HIPCHK(pb, launch_prolong(np, 3, pb->A.n_cells, nullptr, nullptr, nullptr, nullptr, nullptr, &lp, pb->f32, r,
                              zloc, nullptr, st_done, 0, 0, s));
  }  // (small subdomains without the side stream: solved inside the prolongation)
  if (ev1) HIPCHK(pb, hipEventRecord(ev1, s));
  if (side) {
    HIPCHK(pb, hipStreamWaitEvent(s, pb->join_ev, 0));
  } else if (pb->has_coarse) {
    asdg_status ce = enqueue_coarse_solve(pb, st_done, s);
    if (ce != ASDG_OK) return ce;
  }
  LocalParts lp = local_parts(pb);
  if (pb->small && side) {
    lp.part = zloc;
    lp.small = 3;
  }
  HIPCHK(pb, launch_prolong(np, pb->has_coarse ? pb->C.nq : 3, pb->A.n_cells,
                            pb->has_coarse ? pb->ptr<int32_t>(2, pb->o2.pptr) : nullptr,
                            pb->ptr<int32_t>(2, pb->o2.pcol), pb->ptr<double>(2, pb->o2.pval),
                            pb->ptr<double>(3, pb->o3.z0), pb->ptr<void>(3, pb->o3.zl),
                            pb->inv_planned || pb->small ? &lp : nullptr, pb->f32, r, pb->ptr<double>(3, pb->o3.z), red,
                            st_done, iteration ? spmv_parts(pb->n()) : 0, iteration ? vec_parts(pb->n()) : 0, s));
  return ASDG_OK;
}

asdg_status enqueue_iteration(asdg_problem* pb, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const int np = pb->A.np;
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  Reduction* red = pb->ptr<Reduction>(3, pb->o3.red);
  double* x = pb->ptr<double>(3, pb->o3.x);
  double* r = pb->ptr<double>(3, pb->o3.r);
  double* p = pb->ptr<double>(3, pb->o3.p);
  double* q = pb->ptr<double>(3, pb->o3.q);
  double* z = pb->ptr<double>(3, pb->o3.z);
  double* rz2 = pb->ptr<double>(3, pb->o3.rz2);
  HIPCHK(pb, launch_spmv(np, pb->A.n_cells, pb->ptr<int32_t>(0, pb->o0.row_ptr), pb->ptr<int32_t>(0, pb->o0.col),
                         pb->ptr<double>(0, pb->o0.blocks), p, q, red, st, s));
  const bool sweeps = !pb->inv_planned && !pb->small;  // only the sweeps consume yl/zl
  HIPCHK(pb, launch_update_xr(pb->n(), st, red, spmv_parts(pb->n()), rz2, pb->ptr<double>(3, pb->o3.ah), p, q, x,
                              r, sweeps ? pb->ptr<void>(3, pb->o3.yl) : nullptr,
                              sweeps ? pb->ptr<void>(3, pb->o3.zl) : nullptr, pb->f32, s));
  asdg_status e = enqueue_precond(pb, s, st, red, true, ev0, ev1);
  if (e != ASDG_OK) return e;
  HIPCHK(pb, launch_update_p(pb->n(), st, red, prolong_parts(pb->n()), rz2, pb->ptr<double>(3, pb->o3.bh), z, p, 0,
                             s));
  return ASDG_OK;
}

asdg_status read_state(asdg_problem* pb, hipStream_t s, DevState& h) {
  HIPCHK(pb, hipMemcpyAsync(&h, pb->ptr<DevState>(3, pb->o3.st), sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(pb, hipStreamSynchronize(s));
  return ASDG_OK;
}

}  // namespace


namespace {

asdg_status ensure_graph(asdg_problem* pb, int k) {
  if (pb->gexec && pb->g_k == k && !pb->g_timed) return ASDG_OK;
  if (!pb->own_stream) HIPCHK(pb, hipStreamCreateWithFlags(&pb->own_stream, hipStreamNonBlocking));
  pb->drop_graph();
  hipGraph_t g;
  HIPCHK(pb, hipStreamBeginCapture(pb->own_stream, hipStreamCaptureModeThreadLocal));
  asdg_status ce = ASDG_OK;
  for (int i = 0; i < k && ce == ASDG_OK; ++i) ce = enqueue_iteration(pb, pb->own_stream, nullptr, nullptr);
  hipError_t he = hipStreamEndCapture(pb->own_stream, &g);
  if (ce != ASDG_OK) return ce;
  if (he != hipSuccess) FAIL(pb, ASDG_EHIP, std::string("graph capture: ") + hipGetErrorString(he));
  he = hipGraphInstantiate(&pb->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (he != hipSuccess) FAIL(pb, ASDG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(he));
  pb->g_k = k;
  pb->g_timed = 0;
  return ASDG_OK;
}

// ||b - A x||^2 of the internal iterate into DevState::trr: q = A x (q is
// free once the loop has stopped), then the fixed-order sum of the squared
// differences with b (d_b, or the assembled load vector when NULL).
asdg_status enqueue_true_residual(asdg_problem* pb, const double* d_b, hipStream_t s) {
  const int np = pb->A.np;
  const int32_t N = pb->A.n_cells;
  const double* src = d_b ? d_b : pb->ptr<double>(0, pb->o0.rhs);
  double* q = pb->ptr<double>(3, pb->o3.q);
  HIPCHK(pb, launch_spmv(np, N, pb->ptr<int32_t>(0, pb->o0.row_ptr), pb->ptr<int32_t>(0, pb->o0.col),
                         pb->ptr<double>(0, pb->o0.blocks), pb->ptr<double>(3, pb->o3.x), q, nullptr, nullptr, s));
  HIPCHK(pb, launch_true_residual(np, N, pb->ptr<int32_t>(0, pb->o0.perm), src, q,
                                  pb->ptr<Reduction>(3, pb->o3.red) + RED_BB, pb->ptr<DevState>(3, pb->o3.st), s));
  return ASDG_OK;
}

// x = 0, r = b, z = P^{-1} r, p = z on stream s.
asdg_status enqueue_begin(asdg_problem* pb, const double* d_b, const asdg_pcg_opts& o, hipStream_t s) {
  const int np = pb->A.np;
  const int32_t N = pb->A.n_cells;
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  Reduction* red = pb->ptr<Reduction>(3, pb->o3.red);
  const double* src = d_b ? d_b : pb->ptr<double>(0, pb->o0.rhs);
  HIPCHK(pb, launch_permute_in(np, N, pb->ptr<int32_t>(0, pb->o0.perm), src, pb->ptr<double>(3, pb->o3.r),
                               pb->ptr<double>(3, pb->o3.x), pb->ptr<void>(3, pb->o3.yl), pb->ptr<void>(3, pb->o3.zl),
                               pb->f32, red, st, o.rtol, o.max_iter, s));
  asdg_status e = enqueue_precond(pb, s, st, red, false, nullptr, nullptr);
  if (e != ASDG_OK) return e;
  HIPCHK(pb, launch_update_p(pb->n(), st, red, prolong_parts(pb->n()), pb->ptr<double>(3, pb->o3.rz2),
                             pb->ptr<double>(3, pb->o3.bh), pb->ptr<double>(3, pb->o3.z), pb->ptr<double>(3, pb->o3.p),
                             1, s));
  return ASDG_OK;
}

// Reads the alpha/beta history on stream s (never the legacy stream: another
// thread may be capturing a graph, which forbids implicit legacy-stream syncs).
asdg_status fill_stats(asdg_problem* pb, const DevState& h, double solve_ms, double t_local, int n_local,
                       asdg_pcg_stats* stats, hipStream_t s) {
  if (!stats) return ASDG_OK;
  std::memset(stats, 0, sizeof(*stats));
  stats->iterations = h.it;
  stats->converged = h.status == 1;
  stats->rel_res = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
  stats->t_solve_ms = solve_ms;
  stats->t_local_ms = t_local;
  stats->n_local = n_local;
  stats->failed_subdomain = -2;
  stats->true_rel_res = h.bb > 0 ? std::sqrt(h.trr / h.bb) : 0.0;
  stats->t_assemble_ms = pb->t_assemble_ms;
  stats->t_factor_ms = pb->t_factor_ms;
  stats->t_coarse_ms = pb->t_coarse_host_ms + pb->t_coarse_dev_ms;
  const int ka = std::min(h.it, HIST);
  if (ka >= 1) {
    std::vector<double> al(ka), be(std::max(ka - 1, 0));
    HIPCHK(pb, hipMemcpyAsync(al.data(), pb->ptr<double>(3, pb->o3.ah), 8 * ka, hipMemcpyDeviceToHost, s));
    if (ka > 1)
      HIPCHK(pb, hipMemcpyAsync(be.data(), pb->ptr<double>(3, pb->o3.bh), 8 * (ka - 1), hipMemcpyDeviceToHost, s));
    HIPCHK(pb, hipStreamSynchronize(s));
    std::vector<double> d(ka), off(std::max(ka - 1, 0));
    d[0] = 1.0 / al[0];
    for (int j = 1; j < ka; ++j) d[j] = 1.0 / al[j] + be[j - 1] / al[j - 1];
    for (int j = 0; j + 1 < ka; ++j) off[j] = std::sqrt(std::max(be[j], 0.0)) / al[j];
    tridiag_extremes(d, off, stats->lambda_min, stats->lambda_max);
  }
  return ASDG_OK;
}

asdg_status status_of(asdg_problem* pb, const DevState& h) {
  if (h.status == 4) FAIL(pb, ASDG_EHIP, "local-solve wait budget exhausted");
  if (h.status == 3) FAIL(pb, ASDG_EBREAKDOWN, "PCG breakdown (p.Ap <= 0 or NaN)");
  if (h.status == 2) FAIL(pb, ASDG_ENOCONV, "maximum number of iterations reached");
  return ASDG_OK;
}

asdg_status enqueue_state_copy(asdg_problem* pb, hipStream_t s) {
  if (!pb->h_state) {
    void* p = nullptr;
    HIPCHK(pb, hipHostMalloc(&p, sizeof(DevState), hipHostMallocDefault));
    pb->h_state = (DevState*)p;
  }
  if (!pb->chunk_ev) HIPCHK(pb, hipEventCreateWithFlags(&pb->chunk_ev, hipEventDisableTiming));
  HIPCHK(pb, hipMemcpyAsync(pb->h_state, pb->ptr<DevState>(3, pb->o3.st), sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(pb, hipEventRecord(pb->chunk_ev, s));
  pb->chunk_in_flight = true;
  return ASDG_OK;
}

}  // namespace

extern "C" {

asdg_status asdg_pcg_begin(asdg_problem* pb, const double* d_b, const asdg_pcg_opts* opts, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (pb->stage < 4 || !pb->coarse_ready) FAIL(pb, ASDG_ESTATE, "asdg_pcg_begin before asdg_factor/asdg_setup_coarse");
  if (pb->chunk_in_flight) FAIL(pb, ASDG_ESTATE, "a chunk of the previous solve is still in flight");
  asdg_pcg_opts o{1e-8, 20000, 16, 1, 0};
  if (opts) o = *opts;
  if (!(o.rtol >= 0.0) || o.max_iter < 1 || o.check_every < 1) FAIL(pb, ASDG_EINVAL, "invalid PCG options");
  o.use_graph = 1;
  o.time_kernels = 0;
  asdg_status e = ensure_graph(pb, o.check_every);
  if (e != ASDG_OK) return e;
  hipStream_t s = (hipStream_t)stream;
  if (!pb->t0) {
    HIPCHK(pb, hipEventCreate(&pb->t0));
    HIPCHK(pb, hipEventCreate(&pb->t1));
  }
  HIPCHK(pb, hipEventRecord(pb->t0, s));
  e = enqueue_begin(pb, d_b, o, s);
  if (e != ASDG_OK) return e;
  pb->aopts = o;
  pb->solve_b = d_b;
  pb->solve_open = true;
  pb->hs = DevState{};
  return enqueue_state_copy(pb, s);
}

asdg_status asdg_pcg_step(asdg_problem* pb, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (!pb->solve_open) FAIL(pb, ASDG_ESTATE, "no open solve");
  if (pb->chunk_in_flight) FAIL(pb, ASDG_ESTATE, "previous chunk not yet observed by asdg_pcg_poll");
  if (pb->hs.done) return ASDG_OK;
  HIPCHK(pb, hipGraphLaunch(pb->gexec, (hipStream_t)stream));
  return enqueue_state_copy(pb, (hipStream_t)stream);
}

asdg_status asdg_pcg_poll(asdg_problem* pb, int32_t* chunk_done, int32_t* solve_done, int32_t* iterations) {
  if (!pb) return ASDG_EINVAL;
  if (!pb->solve_open) FAIL(pb, ASDG_ESTATE, "no open solve");
  if (pb->chunk_in_flight) {
    hipError_t q = hipEventQuery(pb->chunk_ev);
    if (q == hipErrorNotReady) {
      if (chunk_done) *chunk_done = 0;
      if (solve_done) *solve_done = 0;
      if (iterations) *iterations = pb->hs.it;
      return ASDG_OK;
    }
    if (q != hipSuccess) FAIL(pb, ASDG_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    pb->hs = *pb->h_state;
    pb->chunk_in_flight = false;
  }
  if (chunk_done) *chunk_done = 1;
  if (solve_done) *solve_done = pb->hs.done ? 1 : 0;
  if (iterations) *iterations = pb->hs.it;
  return ASDG_OK;
}

asdg_status asdg_pcg_finish(asdg_problem* pb, double* d_x, asdg_pcg_stats* stats, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (!pb->solve_open) FAIL(pb, ASDG_ESTATE, "no open solve");
  if (pb->chunk_in_flight || !pb->hs.done) FAIL(pb, ASDG_ESTATE, "solve not finished (poll until solve_done)");
  if (!d_x) FAIL(pb, ASDG_EINVAL, "d_x is null");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(pb, launch_unpermute_out(pb->A.np, pb->A.n_cells, pb->ptr<int32_t>(0, pb->o0.perm),
                                  pb->ptr<double>(3, pb->o3.x), d_x, s));
  HIPCHK(pb, hipEventRecord(pb->t1, s));
  pb->solve_open = false;
  asdg_status e = enqueue_true_residual(pb, pb->solve_b, s);
  if (e != ASDG_OK) return e;
  DevState h;
  e = read_state(pb, s, h);
  if (e != ASDG_OK) return e;
  float ms = 0.f;
  HIPCHK(pb, hipEventElapsedTime(&ms, pb->t0, pb->t1));
  e = fill_stats(pb, h, ms, 0.0, 0, stats, (hipStream_t)stream);
  if (e != ASDG_OK) return e;
  return status_of(pb, pb->hs);
}

asdg_status asdg_plan(asdg_problem* pb, asdg_precision precision, int32_t q, const int32_t* coarse_of_cell,
                      const asdg_mesh* coarse_mesh, size_t bytes[4]) {
  if (!pb) return ASDG_EINVAL;
  if (pb->stage < 1) FAIL(pb, ASDG_ESTATE, "asdg_plan before asdg_assemble");
  HostThreadCap cap(pb->host_threads);
  if (precision != ASDG_FP64 && precision != ASDG_FP32_LOCAL) FAIL(pb, ASDG_EINVAL, "unknown precision");
  if (!bytes) FAIL(pb, ASDG_EINVAL, "bytes is null");
  if (q < 0 || q > pb->A.p) FAIL(pb, ASDG_EINVAL, "coarse degree q must satisfy 1 <= q <= p (or 0: no coarse level)");
  if (pb->A.dim == 2 && pb->A.p >= 5 && q != 0 && q != 1 && q != pb->A.p)
    FAIL(pb, ASDG_EINVAL, "for p >= 5 the coarse degree q must be 1 or p");
  pb->drop_graph();
  pb->stage = 1;
  pb->coarse_ready = false;
  pb->f32 = precision == ASDG_FP32_LOCAL;
  pb->has_coarse = q > 0;
  pb->n0 = 0;
  pb->C = Coarse();
  if (pb->has_coarse) {
    if (!coarse_of_cell && !coarse_mesh) FAIL(pb, ASDG_EINVAL, "coarse level needs coarse_of_cell or coarse_mesh");
    MeshView cm{};
    if (coarse_mesh) {
      if (!coarse_mesh->xy || !coarse_mesh->cell_ptr || !coarse_mesh->cell_vertices || coarse_mesh->n_cells < 1)
        FAIL(pb, ASDG_EINVAL, "invalid coarse mesh");
      cm = MeshView{coarse_mesh->n_vertices, coarse_mesh->xy, coarse_mesh->n_cells, coarse_mesh->cell_ptr,
                    coarse_mesh->cell_vertices};
    }
    std::string e;
    const double tc = wall_ms();
    if (pb->A.dim == 3) {
      if (coarse_mesh) FAIL(pb, ASDG_EINVAL, "tetrahedral meshes take nested agglomerates (coarse_of_cell)");
      e = build_coarse_tet(pb->tet.view(), pb->A, q, coarse_of_cell, pb->C);
    } else {
      e = build_coarse(pb->fine.view(), pb->A, q, coarse_of_cell, coarse_mesh ? &cm : nullptr, pb->C);
    }
    if (!e.empty()) FAIL(pb, ASDG_EINVAL, e);
    pb->n0 = pb->C.n_coarse * pb->C.nq;
    plan_coarse_factor(pb);
    pb->t_coarse_host_ms = wall_ms() - tc;
  }
  if (pb->local_inverse && pb->tile_req == 32)
    FAIL(pb, ASDG_EINVAL, "explicit local inverses are stored in 64-row tiles (ASDG_TUNE_TILE 32 needs the sweeps)");
  pb->tile = pb->tile_req ? pb->tile_req : TILE;
  plan_local(pb);
  pb->inv_planned = pb->local_inverse && !pb->small;
  // with the automatic edge, room for the layouts of both edges (the 32-row
  // layout never stores more tile words, it has more tiles and tasks), so
  // that the autotuner can switch between them in the bound buffers
  pb->tile_search = pb->tile_req == 0 && !pb->inv_planned && !pb->small;
  int64_t res_tiles = pb->n_tiles, res_sweeps = (int64_t)pb->trsv_tasks.size();
  int64_t res_words = pb->n_tiles * pb->tile * pb->tile;
  if (pb->tile_search) {
    for (int t : {32, 64}) {
      int64_t nt = 0, ns = 0;
      local_counts(pb, t, nt, ns);
      res_tiles = std::max(res_tiles, nt);
      res_sweeps = std::max(res_sweeps, ns);
      res_words = std::max(res_words, nt * t * t);
    }
  }
  pb->inv_tasks.clear();
  if (pb->inv_planned) {
    // X = L^{-1} tasks (i, j, b), j <= b: longest path to the end first, so
    // every X_kj with k < b precedes X_bj
    pb->inv_tasks = order_tasks(pb->subs, inverse_levels, pb->task_chunk);
  }
  pb->cell_sub.assign(pb->A.n_cells, 0);
  for (int32_t i = 0; i < pb->A.n_sub; ++i)
    for (int32_t c = pb->A.sub_ptr[i]; c < pb->A.sub_ptr[i + 1]; ++c) pb->cell_sub[c] = i;

  const Assembled& A = pb->A;
  const int64_t N = A.n_cells, n = pb->n(), nnzb = A.row_ptr[N];
  const size_t w = pb->f32 ? 4 : 8;
  Layout L0, L1, L2, L3;
  pb->o0.row_ptr = L0.add(4 * (N + 1));
  pb->o0.col = L0.add(4 * nnzb);
  pb->o0.blocks = L0.add(8 * nnzb * A.np * A.np);
  pb->o0.rhs = L0.add(8 * n);
  pb->o0.perm = L0.add(4 * N);
  pb->o0.cell_sub = L0.add(4 * N);
  pb->o1.tiles = L1.add(pb->small ? (size_t)pb->small_words * w : (size_t)res_words * w);
  pb->o1.subs = L1.add(sizeof(SubDesc) * pb->subs.size());
  pb->o1.chol = L1.add(sizeof(int4) * (size_t)res_tiles);
  pb->o1.trsv = L1.add(sizeof(int4) * (size_t)res_sweeps);
  pb->o1.meta = L1.add(sizeof(int4) * (size_t)res_tiles);
  if (pb->inv_planned) {
    pb->o1.xtiles = L1.add((size_t)pb->n_tiles * TILE * TILE * w);
    pb->o1.inv = L1.add(sizeof(int4) * pb->inv_tasks.size());
    pb->o1.colt = L1.add(sizeof(int4) * pb->col_tasks.size());
  }
  pb->o1.subt = L1.add(sizeof(int4) * std::max<size_t>(1, pb->sub_tasks.size()));
  if (pb->has_coarse) {
    const Coarse& C = pb->C;
    pb->o2.pptr = L2.add(4 * (N + 1));
    pb->o2.pcol = L2.add(4 * C.col.size());
    pb->o2.pval = L2.add(8 * C.val.size());
    pb->o2.tptr = L2.add(4 * C.tptr.size());
    pb->o2.tcell = L2.add(4 * C.tcell.size());
    pb->o2.tblk = L2.add(4 * C.tblk.size());
    pb->o2.ctiles = L2.add(8 * pb->ctiles_host.size());
    pb->o2.csub = L2.add(sizeof(SubDesc));
    pb->o2.cchol = L2.add(sizeof(int4) * pb->cchol_tasks.size());
    pb->o2.ctrsv = L2.add(sizeof(int4) * pb->ctrsv_tasks.size());
    if (pb->coarse_dense) {
      pb->o2.cS = L2.add(8 * pb->ctiles_host.size());
      pb->o2.cX = L2.add(8 * pb->ctiles_host.size());
      pb->o2.cinv = pb->coarse_packed ? 0 : L2.add(8 * (size_t)pb->n0 * pb->n0);
      pb->o2.cmeta = L2.add(sizeof(int4) * pb->cmeta.size());
      pb->o2.cinvt = L2.add(sizeof(int4) * pb->cinv_tasks.size());
    }
  } else {
    L2.add(256);
  }
  const int64_t n0 = std::max<int32_t>(pb->n0, 1);
  pb->o3.x = L3.add(8 * n);
  pb->o3.r = L3.add(8 * n);
  pb->o3.p = L3.add(8 * n);
  pb->o3.q = L3.add(8 * n);
  pb->o3.z = L3.add(8 * n);
  pb->o3.yl = L3.add(w * n);
  pb->o3.zl = L3.add(w * n);
  pb->o3.r0 = L3.add(8 * n0 * (pb->has_coarse ? pb->rsplits : 1));
  pb->o3.y0 = L3.add(8 * n0);
  pb->o3.z0 = L3.add(8 * n0);
  pb->o3.cpart = L3.add(pb->has_coarse && pb->coarse_packed ? 8 * 2 * TILE * (size_t)pb->n_ctiles : 0);
  pb->o3.red = L3.add(sizeof(Reduction) * N_RED);
  pb->o3.st = L3.add(sizeof(DevState));
  pb->o3.rz2 = L3.add(16);
  pb->o3.ah = L3.add(8 * (size_t)HIST);
  pb->o3.bh = L3.add(8 * (size_t)HIST);
  pb->o3.flags = L3.add(4 * (size_t)std::max<int64_t>(res_tiles, pb->n_ctiles));
  pb->o3.trace = L3.add(3 * 8 * (size_t)res_sweeps);
  pb->o3.part = L3.add(pb->inv_planned ? (size_t)pb->n_tiles * 2 * TILE * w : 0);
  pb->bytes[0] = L0.size;
  pb->bytes[1] = L1.size;
  pb->bytes[2] = L2.size;
  pb->bytes[3] = L3.size;
  for (int i = 0; i < 4; ++i) bytes[i] = pb->bytes[i];
  pb->stage = 2;
  return ASDG_OK;
}

asdg_status asdg_bind(asdg_problem* pb, void* const d_buf[4], const size_t sizes[4], void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (pb->stage < 2) FAIL(pb, ASDG_ESTATE, "asdg_bind before asdg_plan");
  if (!d_buf || !sizes) FAIL(pb, ASDG_EINVAL, "null buffer list");
  for (int i = 0; i < 4; ++i) {
    if (!d_buf[i]) FAIL(pb, ASDG_EINVAL, "null device buffer");
    if (sizes[i] < pb->bytes[i]) FAIL(pb, ASDG_ENOMEM, "device buffer " + std::to_string(i) + " too small");
    if (((uintptr_t)d_buf[i]) & 255) FAIL(pb, ASDG_EINVAL, "device buffer not 256-byte aligned");
  }
  pb->drop_graph();
  for (int i = 0; i < 4; ++i) pb->buf[i] = (char*)d_buf[i];
  int dev = 0;
  HIPCHK(pb, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(pb, hipGetDeviceProperties(&prop, dev));
  pb->n_cu = std::max(1, prop.multiProcessorCount);
  pb->arch = prop.gcnArchName;
  if (!pb->side_stream) {
    HIPCHK(pb, hipStreamCreateWithFlags(&pb->side_stream, hipStreamNonBlocking));
    HIPCHK(pb, hipEventCreateWithFlags(&pb->fork_ev, hipEventDisableTiming));
    HIPCHK(pb, hipEventCreateWithFlags(&pb->join_ev, hipEventDisableTiming));
  }
  hipStream_t s = (hipStream_t)stream;
  const Assembled& A = pb->A;
  auto up = [&](int b, size_t off, const void* src, size_t nbytes) {
    return nbytes ? hipMemcpyAsync(pb->buf[b] + off, src, nbytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  HIPCHK(pb, up(0, pb->o0.row_ptr, A.row_ptr.data(), 4 * A.row_ptr.size()));
  HIPCHK(pb, up(0, pb->o0.col, A.col_idx.data(), 4 * A.col_idx.size()));
  HIPCHK(pb, up(0, pb->o0.blocks, A.blocks.data(), 8 * A.blocks.size()));  // row-major blocks, as on the device
  HIPCHK(pb, up(0, pb->o0.rhs, pb->rhs_caller.data(), 8 * pb->rhs_caller.size()));
  HIPCHK(pb, up(0, pb->o0.perm, A.perm.data(), 4 * A.perm.size()));
  HIPCHK(pb, up(0, pb->o0.cell_sub, pb->cell_sub.data(), 4 * pb->cell_sub.size()));
  if (pb->inv_planned) {
    HIPCHK(pb, up(1, pb->o1.inv, pb->inv_tasks.data(), sizeof(int4) * pb->inv_tasks.size()));
    HIPCHK(pb, up(1, pb->o1.colt, pb->col_tasks.data(), sizeof(int4) * pb->col_tasks.size()));
  }
  if (!pb->sub_tasks.empty()) HIPCHK(pb, up(1, pb->o1.subt, pb->sub_tasks.data(), sizeof(int4) * pb->sub_tasks.size()));
  HIPCHK(pb, up(1, pb->o1.subs, pb->subs.data(), sizeof(SubDesc) * pb->subs.size()));
  HIPCHK(pb, up(1, pb->o1.chol, pb->chol_tasks.data(), sizeof(int4) * pb->chol_tasks.size()));
  HIPCHK(pb, up(1, pb->o1.trsv, pb->trsv_tasks.data(), sizeof(int4) * pb->trsv_tasks.size()));
  HIPCHK(pb, up(1, pb->o1.meta, pb->tile_meta.data(), sizeof(int4) * pb->tile_meta.size()));
  if (pb->has_coarse) {
    const Coarse& C = pb->C;
    HIPCHK(pb, up(2, pb->o2.pptr, C.ptr.data(), 4 * C.ptr.size()));
    HIPCHK(pb, up(2, pb->o2.pcol, C.col.data(), 4 * C.col.size()));
    HIPCHK(pb, up(2, pb->o2.pval, C.val.data(), 8 * C.val.size()));
    HIPCHK(pb, up(2, pb->o2.tptr, C.tptr.data(), 4 * C.tptr.size()));
    HIPCHK(pb, up(2, pb->o2.tcell, C.tcell.data(), 4 * C.tcell.size()));
    HIPCHK(pb, up(2, pb->o2.tblk, C.tblk.data(), 4 * C.tblk.size()));
    HIPCHK(pb, up(2, pb->o2.csub, &pb->csub, sizeof(SubDesc)));
    HIPCHK(pb, up(2, pb->o2.cchol, pb->cchol_tasks.data(), sizeof(int4) * pb->cchol_tasks.size()));
    HIPCHK(pb, up(2, pb->o2.ctrsv, pb->ctrsv_tasks.data(), sizeof(int4) * pb->ctrsv_tasks.size()));
    if (pb->coarse_dense) {
      HIPCHK(pb, up(2, pb->o2.cmeta, pb->cmeta.data(), sizeof(int4) * pb->cmeta.size()));
      HIPCHK(pb, up(2, pb->o2.cinvt, pb->cinv_tasks.data(), sizeof(int4) * pb->cinv_tasks.size()));
    }
  }
  HIPCHK(pb, launch_fill_i32(pb->ptr<int32_t>(3, pb->o3.red), (int64_t)(sizeof(Reduction) * N_RED / 4), 0, s));
  HIPCHK(pb, hipStreamSynchronize(s));
  pb->stage = 3;
  pb->coarse_ready = false;
  return ASDG_OK;
}

// Work-groups per compute unit of the Cholesky launch by default: the
// kernel's occupancy (eight waves per CU: two work-groups of four waves for
// 64-row tiles, eight of one wave for 32-row tiles).
static int chol_occupancy(int tile) { return tile == 32 ? 8 : 2; }

// Schedules of the local factorisation (1 tile tasks, 2 one work-group per
// subdomain) and of the formation of X = L^{-1} (1 tile tasks, 2 one
// work-group per block column). The schedules without waits run their
// products faster, the tile tasks spread a large subdomain over many
// work-groups; the automatic choice compares the largest task of the
// coarse-grained schedule with an even share of all products over the
// work-groups that fit on the device.
// Cholesky: subdomain tasks when the largest subdomain (about nb^3/6 tile
// products) is at most 1.5 times that share (measured on 512 subdomains
// whose largest is 1.65 times the mean: the tile tasks are 6% faster).
static int factor_schedule(const asdg_problem* pb) {
  if (pb->factor_sched == 1 || pb->factor_sched == 2) return pb->factor_sched;
  double total = 0.0, largest = 0.0;
  for (const SubDesc& d : pb->subs) {
    const double w = (double)d.nb * d.nb * d.nb;
    total += w;
    largest = std::max(largest, w);
  }
  const int per_cu = pb->chol_per_cu > 0 ? pb->chol_per_cu : chol_occupancy(pb->tile);
  const double slots = (double)pb->n_cu * per_cu;
  return largest <= 1.5 * total / slots ? 2 : 1;
}

// X = L^{-1}: column tasks when the largest column (m(m+3)/2 tile products
// for the m block rows below its diagonal) is at most twice the share (at
// that size the column tasks are 20-35% faster than the tile tasks).
static int inverse_schedule(const asdg_problem* pb) {
  if (pb->inv_sched == 1 || pb->inv_sched == 2) return pb->inv_sched;
  double total = 0.0, largest = 0.0;
  for (const SubDesc& d : pb->subs)
    for (int m = 0; m < d.nb; ++m) {
      const double w = 0.5 * m * (m + 3);
      total += w;
      largest = std::max(largest, w);
    }
  const int per_cu = pb->inv_per_cu > 0 ? pb->inv_per_cu : (pb->f32 ? 4 : 2);
  const double slots = (double)pb->n_cu * per_cu;
  return largest <= 2.0 * total / slots ? 2 : 1;
}

static asdg_status run_cholesky(asdg_problem* pb, hipStream_t s, int f32, int tile, int per_sub, int32_t n_tasks,
                                const int4* tasks, const SubDesc* subs, void* tiles, int64_t n_tiles, int coarse) {
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  int32_t* flags = pb->ptr<int32_t>(3, pb->o3.flags);
  if (!per_sub) HIPCHK(pb, launch_fill_i32(flags, n_tiles, 0, s));
  HIPCHK(pb, launch_reset_queues(st, s));
  const int per_cu = pb->chol_per_cu > 0 ? pb->chol_per_cu : chol_occupancy(tile);
  int64_t gmax = pb->chol_grid > 0 ? pb->chol_grid : (int64_t)pb->n_cu * per_cu;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n_tasks, gmax));
  HIPCHK(pb, launch_cholesky(f32, tile, per_sub, n_tasks, tasks, subs, tiles, flags, st, &st->q_chol, grid, s));
  DevState h;
  asdg_status e = read_state(pb, s, h);
  if (e != ASDG_OK) return e;
  if (h.abort) FAIL(pb, ASDG_EHIP, "factorisation wait budget exhausted");
  if (h.chol_fail != 0x7fffffff) {
    pb->failed_sub = coarse ? -1 : h.chol_fail;
    FAIL(pb, ASDG_ENOTSPD, coarse ? "coarse matrix A_0 is not positive definite"
                                  : "local matrix of subdomain " + std::to_string(h.chol_fail) +
                                        " is not positive definite");
  }
  return ASDG_OK;
}

asdg_status asdg_factor(asdg_problem* pb, void* stream) {
  if (!pb) return ASDG_EINVAL;
  WallTimer timer(pb->t_factor_ms);
  if (pb->stage < 3) FAIL(pb, ASDG_ESTATE, "asdg_factor before asdg_bind");
  hipStream_t s = (hipStream_t)stream;
  pb->failed_sub = -2;
  pb->stage = 3;
  if (pb->small) {
    DevState* st = pb->ptr<DevState>(3, pb->o3.st);
    HIPCHK(pb, launch_reset_queues(st, s));
    HIPCHK(pb, launch_small_inverse(pb->f32, pb->A.n_sub, pb->A.np, pb->max_n, pb->ptr<SubDesc>(1, pb->o1.subs),
                                    pb->ptr<int32_t>(0, pb->o0.row_ptr), pb->ptr<int32_t>(0, pb->o0.col),
                                    pb->ptr<double>(0, pb->o0.blocks), pb->ptr<void>(1, pb->o1.tiles), st, s));
    DevState h;
    asdg_status e = read_state(pb, s, h);
    if (e != ASDG_OK) return e;
    if (h.chol_fail != 0x7fffffff) {
      pb->failed_sub = h.chol_fail;
      FAIL(pb, ASDG_ENOTSPD, "local matrix of subdomain " + std::to_string(h.chol_fail) + " is not positive definite");
    }
    pb->stage = 4;
    return ASDG_OK;
  }
  if (pb->tasks_dirty) {
    // reordered task lists (same size); the status read below completes the copies
    HIPCHK(pb, hipMemcpyAsync(pb->buf[1] + pb->o1.chol, pb->chol_tasks.data(), sizeof(int4) * pb->chol_tasks.size(),
                              hipMemcpyHostToDevice, s));
    if (pb->inv_planned) {
      HIPCHK(pb, hipMemcpyAsync(pb->buf[1] + pb->o1.inv, pb->inv_tasks.data(), sizeof(int4) * pb->inv_tasks.size(),
                                hipMemcpyHostToDevice, s));
      HIPCHK(pb, hipMemcpyAsync(pb->buf[1] + pb->o1.colt, pb->col_tasks.data(), sizeof(int4) * pb->col_tasks.size(),
                                hipMemcpyHostToDevice, s));
    }
    pb->tasks_dirty = false;
  }
  HIPCHK(pb, launch_gather_tiles(pb->A.np, pb->tile, (int32_t)pb->n_tiles, pb->ptr<int4>(1, pb->o1.meta),
                                 pb->ptr<SubDesc>(1, pb->o1.subs), pb->ptr<int32_t>(0, pb->o0.row_ptr),
                                 pb->ptr<int32_t>(0, pb->o0.col), pb->ptr<double>(0, pb->o0.blocks),
                                 pb->ptr<void>(1, pb->o1.tiles), pb->f32, s));
  const bool per_sub = factor_schedule(pb) == 2;
  asdg_status e = per_sub ? run_cholesky(pb, s, pb->f32, pb->tile, 1, (int32_t)pb->sub_tasks.size(),
                                         pb->ptr<int4>(1, pb->o1.subt), pb->ptr<SubDesc>(1, pb->o1.subs),
                                         pb->ptr<void>(1, pb->o1.tiles), pb->n_tiles, 0)
                          : run_cholesky(pb, s, pb->f32, pb->tile, 0, (int32_t)pb->chol_tasks.size(),
                                         pb->ptr<int4>(1, pb->o1.chol), pb->ptr<SubDesc>(1, pb->o1.subs),
                                         pb->ptr<void>(1, pb->o1.tiles), pb->n_tiles, 0);
  if (e != ASDG_OK) return e;
  if (pb->inv_planned) {
    DevState* st = pb->ptr<DevState>(3, pb->o3.st);
    const bool cols = inverse_schedule(pb) == 2;
    if (!cols) HIPCHK(pb, launch_fill_i32(pb->ptr<int32_t>(3, pb->o3.flags), pb->n_tiles, 0, s));
    HIPCHK(pb, launch_reset_queues(st, s));
    const int per_cu = pb->inv_per_cu > 0 ? pb->inv_per_cu : (pb->f32 ? 4 : 2);  // default: the occupancy
    const int64_t nt = cols ? (int64_t)pb->col_tasks.size() : (int64_t)pb->inv_tasks.size();
    const int g1 = (int)std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t)pb->n_cu * per_cu));
    const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>(pb->n_tiles, (int64_t)pb->n_cu * per_cu * 4));
    HIPCHK(pb, launch_inverse(pb->f32, cols ? 1 : 0, (int32_t)nt,
                              cols ? pb->ptr<int4>(1, pb->o1.colt) : pb->ptr<int4>(1, pb->o1.inv),
                              (int32_t)pb->n_tiles, pb->ptr<int4>(1, pb->o1.meta), pb->ptr<SubDesc>(1, pb->o1.subs),
                              pb->ptr<void>(1, pb->o1.tiles), pb->ptr<void>(1, pb->o1.xtiles),
                              pb->ptr<int32_t>(3, pb->o3.flags), st, &st->q_chol, g1, g2, s));
    DevState h;
    e = read_state(pb, s, h);
    if (e != ASDG_OK) return e;
    if (h.abort) FAIL(pb, ASDG_EHIP, "inverse formation wait budget exhausted");
  }
  pb->stage = 4;
  return ASDG_OK;
}

asdg_status asdg_setup_coarse(asdg_problem* pb, void* stream) {
  if (!pb) return ASDG_EINVAL;
  WallTimer timer(pb->t_coarse_dev_ms);
  if (pb->stage < 3) FAIL(pb, ASDG_ESTATE, "asdg_setup_coarse before asdg_bind");
  pb->coarse_ready = false;
  if (!pb->has_coarse) {
    pb->coarse_ready = true;
    return ASDG_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(pb, hipMemcpyAsync(pb->buf[2] + pb->o2.ctiles, pb->ctiles_host.data(), 8 * pb->ctiles_host.size(),
                            hipMemcpyHostToDevice, s));
  asdg_status e = run_cholesky(pb, s, 0, TILE, 0, (int32_t)pb->cchol_tasks.size(), pb->ptr<int4>(2, pb->o2.cchol),
                               pb->ptr<SubDesc>(2, pb->o2.csub), pb->ptr<void>(2, pb->o2.ctiles), pb->n_ctiles, 1);
  if (e != ASDG_OK) return e;
  if (pb->coarse_dense) {
    // A_0^{-1} = L^{-T} L^{-1} from a copy of the factor (the factor tiles stay exportable), then dense
    DevState* st = pb->ptr<DevState>(3, pb->o3.st);
    HIPCHK(pb, hipMemcpyAsync(pb->buf[2] + pb->o2.cS, pb->buf[2] + pb->o2.ctiles, 8 * pb->ctiles_host.size(),
                              hipMemcpyDeviceToDevice, s));
    HIPCHK(pb, launch_fill_i32(pb->ptr<int32_t>(3, pb->o3.flags), pb->n_ctiles, 0, s));
    HIPCHK(pb, launch_reset_queues(st, s));
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(pb->n_ctiles, (int64_t)pb->n_cu * 2));
    HIPCHK(pb, launch_inverse(0, 0, (int32_t)pb->cinv_tasks.size(), pb->ptr<int4>(2, pb->o2.cinvt),
                              (int32_t)pb->n_ctiles, pb->ptr<int4>(2, pb->o2.cmeta), pb->ptr<SubDesc>(2, pb->o2.csub),
                              pb->ptr<void>(2, pb->o2.cS), pb->ptr<void>(2, pb->o2.cX),
                              pb->ptr<int32_t>(3, pb->o3.flags), st, &st->q_chol, g, g, s));
    if (!pb->coarse_packed)
      HIPCHK(pb, launch_expand_sym(pb->n0, pb->ptr<double>(2, pb->o2.cS), pb->ptr<double>(2, pb->o2.cinv), s));
    DevState h;
    e = read_state(pb, s, h);
    if (e != ASDG_OK) return e;
    if (h.abort) FAIL(pb, ASDG_EHIP, "coarse inverse wait budget exhausted");
  }
  pb->coarse_ready = true;
  return ASDG_OK;
}

asdg_status asdg_pcg_solve(asdg_problem* pb, const double* d_b, double* d_x, const asdg_pcg_opts* opts,
                           asdg_pcg_stats* stats, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (pb->stage < 4 || !pb->coarse_ready) FAIL(pb, ASDG_ESTATE, "asdg_pcg_solve before asdg_factor/asdg_setup_coarse");
  if (!d_x) FAIL(pb, ASDG_EINVAL, "d_x is null");
  if (pb->chunk_in_flight) FAIL(pb, ASDG_ESTATE, "a non-blocking solve is in flight");
  asdg_pcg_opts o{1e-8, 20000, 16, 1, 0};
  if (opts) o = *opts;
  if (!(o.rtol >= 0.0) || o.max_iter < 1 || o.check_every < 1) FAIL(pb, ASDG_EINVAL, "invalid PCG options");
  // HIP events recorded inside a captured graph do not bracket the kernel
  // between them, so kernel timing always uses eager launches
  if (o.time_kernels) o.use_graph = 0;
  hipStream_t s = (hipStream_t)stream;
  const int k = o.check_every;
  if (!pb->t0) {
    HIPCHK(pb, hipEventCreate(&pb->t0));
    HIPCHK(pb, hipEventCreate(&pb->t1));
  }
  while ((int)pb->ev.size() < 2 * k) {
    hipEvent_t e;
    HIPCHK(pb, hipEventCreate(&e));
    pb->ev.push_back(e);
  }
  if (o.use_graph) {
    asdg_status ge = ensure_graph(pb, k);
    if (ge != ASDG_OK) return ge;
  }
  HIPCHK(pb, hipEventRecord(pb->t0, s));
  asdg_status e = enqueue_begin(pb, d_b, o, s);
  if (e != ASDG_OK) return e;
  double t_local = 0.0;
  int n_local = 0;
  DevState h;
  e = read_state(pb, s, h);
  if (e != ASDG_OK) return e;
  while (!h.done) {
    const int it0 = h.it;
    if (o.use_graph) {
      HIPCHK(pb, hipGraphLaunch(pb->gexec, s));
    } else {
      for (int i = 0; i < k; ++i) {
        e = enqueue_iteration(pb, s, o.time_kernels ? pb->ev[2 * i] : nullptr,
                              o.time_kernels ? pb->ev[2 * i + 1] : nullptr);
        if (e != ASDG_OK) return e;
      }
    }
    e = read_state(pb, s, h);
    if (e != ASDG_OK) return e;
    if (o.time_kernels) {
      // the local solve of the iteration that stops does not run
      const int ran = h.it - it0 - (h.done ? 1 : 0);
      for (int i = 0; i < ran && i < k; ++i) {
        float ms = 0.f;
        HIPCHK(pb, hipEventElapsedTime(&ms, pb->ev[2 * i], pb->ev[2 * i + 1]));
        t_local += ms;
        ++n_local;
      }
    }
  }
  HIPCHK(pb, launch_unpermute_out(pb->A.np, pb->A.n_cells, pb->ptr<int32_t>(0, pb->o0.perm),
                                  pb->ptr<double>(3, pb->o3.x), d_x, s));
  HIPCHK(pb, hipEventRecord(pb->t1, s));
  e = enqueue_true_residual(pb, d_b, s);
  if (e != ASDG_OK) return e;
  e = read_state(pb, s, h);
  if (e != ASDG_OK) return e;
  float solve_ms = 0.f;
  HIPCHK(pb, hipEventElapsedTime(&solve_ms, pb->t0, pb->t1));
  e = fill_stats(pb, h, solve_ms, t_local, n_local, stats, s);
  if (e != ASDG_OK) return e;
  return status_of(pb, h);
}

asdg_status asdg_apply(asdg_problem* pb, int32_t what, const double* d_in, double* d_out, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (!d_in || !d_out) FAIL(pb, ASDG_EINVAL, "null vector");
  if (what < 0 || what > 3) FAIL(pb, ASDG_EINVAL, "unknown operator");
  if (what == ASDG_APPLY_OPERATOR && pb->stage < 3) FAIL(pb, ASDG_ESTATE, "apply before asdg_bind");
  if ((what == ASDG_APPLY_LOCAL || what == ASDG_APPLY_PRECOND) && pb->stage < 4)
    FAIL(pb, ASDG_ESTATE, "apply before asdg_factor");
  if ((what == ASDG_APPLY_COARSE || what == ASDG_APPLY_PRECOND) && !pb->coarse_ready)
    FAIL(pb, ASDG_ESTATE, "apply before asdg_setup_coarse");
  hipStream_t s = (hipStream_t)stream;
  const int np = pb->A.np;
  const int32_t N = pb->A.n_cells;
  DevState* st = pb->ptr<DevState>(3, pb->o3.st);
  double* r = pb->ptr<double>(3, pb->o3.r);
  double* q = pb->ptr<double>(3, pb->o3.q);
  double* z = pb->ptr<double>(3, pb->o3.z);
  int32_t* perm = pb->ptr<int32_t>(0, pb->o0.perm);
  HIPCHK(pb, launch_permute_in(np, N, perm, d_in, r, nullptr, pb->ptr<void>(3, pb->o3.yl), pb->ptr<void>(3, pb->o3.zl),
                               pb->f32, nullptr, nullptr, 0.0, 0, s));
  HIPCHK(pb, launch_reset_queues(st, s));
  if (what == ASDG_APPLY_OPERATOR) {
    HIPCHK(pb, launch_spmv(np, N, pb->ptr<int32_t>(0, pb->o0.row_ptr), pb->ptr<int32_t>(0, pb->o0.col),
                           pb->ptr<double>(0, pb->o0.blocks), r, q, nullptr, nullptr, s));
    HIPCHK(pb, launch_unpermute_out(np, N, perm, q, d_out, s));
  } else {
    const bool loc = what != ASDG_APPLY_COARSE, crs = what != ASDG_APPLY_LOCAL && pb->has_coarse;
    if (crs)
      HIPCHK(pb, launch_restrict(np, pb->C.nq, pb->C.n_coarse, pb->rsplits, pb->ptr<int32_t>(2, pb->o2.tptr),
                                 pb->ptr<int32_t>(2, pb->o2.tcell), pb->ptr<int32_t>(2, pb->o2.tblk),
                                 pb->ptr<double>(2, pb->o2.pval), r, pb->ptr<double>(3, pb->o3.r0),
                                 pb->coarse_dense ? nullptr : pb->ptr<double>(3, pb->o3.y0),
                                 pb->coarse_dense ? nullptr : pb->ptr<double>(3, pb->o3.z0), nullptr, s));
    if (loc && !pb->small) {  // (small subdomains: the local solves happen inside the prolongation)
      asdg_status le = enqueue_local(pb, s, nullptr);
      if (le != ASDG_OK) return le;
    }
    if (crs) {
      asdg_status ce = enqueue_coarse_solve(pb, nullptr, s);
      if (ce != ASDG_OK) return ce;
    }
    const LocalParts lp = local_parts(pb);
    HIPCHK(pb, launch_prolong(np, crs ? pb->C.nq : 3, N, crs ? pb->ptr<int32_t>(2, pb->o2.pptr) : nullptr,
                              pb->ptr<int32_t>(2, pb->o2.pcol), pb->ptr<double>(2, pb->o2.pval),
                              pb->ptr<double>(3, pb->o3.z0), loc ? pb->ptr<void>(3, pb->o3.zl) : nullptr,
                              loc && (pb->inv_planned || pb->small) ? &lp : nullptr, pb->f32, r, z, nullptr, nullptr,
                              0, 0, s));
    HIPCHK(pb, launch_unpermute_out(np, N, perm, z, d_out, s));
  }
  DevState h;
  asdg_status e = read_state(pb, s, h);
  if (e != ASDG_OK) return e;
  if (h.abort) FAIL(pb, ASDG_EHIP, "wait budget exhausted");
  return ASDG_OK;
}

asdg_status asdg_apply_operator_static(asdg_problem* pb, const double* d_in, double* d_out, void* stream) {
  if (!pb) return ASDG_EINVAL;
  if (!d_in || !d_out) FAIL(pb, ASDG_EINVAL, "null vector");
  if (pb->stage < 3) FAIL(pb, ASDG_ESTATE, "apply before asdg_bind");
  if (pb->n() > kStaticMaxDofs)
    FAIL(pb, ASDG_EINVAL, "asdg_apply_operator_static takes at most " + std::to_string(kStaticMaxDofs) +
                              " DoFs (problem has " + std::to_string(pb->n()) + ")");
  double* ws = nullptr;
  HIPCHK(pb, static_scratch(&ws));
  hipStream_t s = (hipStream_t)stream;
  const int np = pb->A.np;
  const int32_t N = pb->A.n_cells;
  const int32_t* perm = pb->ptr<int32_t>(0, pb->o0.perm);
  double* in_w = ws;
  double* out_w = ws + pb->n();
  HIPCHK(pb, launch_permute_in(np, N, perm, d_in, in_w, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0.0, 0, s));
  HIPCHK(pb, launch_spmv(np, N, pb->ptr<int32_t>(0, pb->o0.row_ptr), pb->ptr<int32_t>(0, pb->o0.col),
                         pb->ptr<double>(0, pb->o0.blocks), in_w, out_w, nullptr, nullptr, s));
  HIPCHK(pb, launch_unpermute_out(np, N, perm, out_w, d_out, s));
  return ASDG_OK;
}

asdg_status asdg_info(const asdg_problem* pb, int64_t info[8]) {
  if (!pb || !info) return ASDG_EINVAL;
  if (pb->stage < 1) return ASDG_ESTATE;
  info[0] = pb->A.n_cells;
  info[1] = pb->A.np;
  info[2] = (int64_t)pb->A.n_cells * pb->A.np;
  info[3] = pb->A.n_sub;
  info[4] = pb->n0;
  info[5] = pb->A.row_ptr.empty() ? 0 : pb->A.row_ptr.back();
  info[6] = pb->max_n;
  info[7] = pb->tile;
  return ASDG_OK;
}

asdg_status asdg_export_rhs(const asdg_problem* pb, double* b) {
  if (!pb || !b) return ASDG_EINVAL;
  if (pb->stage < 1) return ASDG_ESTATE;
  std::memcpy(b, pb->rhs_caller.data(), 8 * pb->rhs_caller.size());
  return ASDG_OK;
}

asdg_status asdg_export_operator(const asdg_problem* pb, int64_t* rows, int64_t* cols, double* vals) {
  if (!pb || !rows || !cols || !vals) return ASDG_EINVAL;
  if (pb->stage < 1) return ASDG_ESTATE;
  const Assembled& A = pb->A;
  const int np = A.np;
  int64_t o = 0;
  for (int32_t r = 0; r < A.n_cells; ++r)
    for (int32_t k = A.row_ptr[r]; k < A.row_ptr[r + 1]; ++k) {
      const int64_t cr = A.perm[r], cc = A.perm[A.col_idx[k]];
      const double* B = &A.blocks[(size_t)k * np * np];
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b, ++o) {
          rows[o] = cr * np + a;
          cols[o] = cc * np + b;
          vals[o] = B[a * np + b];
        }
    }
  return ASDG_OK;
}

asdg_status asdg_export_coarse(const asdg_problem* pb, double* a0) {
  if (!pb || !a0) return ASDG_EINVAL;
  if (pb->stage < 2 || !pb->has_coarse) return ASDG_ESTATE;
  std::memcpy(a0, pb->C.a0.data(), 8 * pb->C.a0.size());
  return ASDG_OK;
}

int32_t asdg_failed_subdomain(const asdg_problem* pb) { return pb ? pb->failed_sub : -2; }

asdg_status asdg_export_factor_tiles(asdg_problem* pb, int32_t sub, void* out, size_t out_bytes) {
  if (!pb || !out) return ASDG_EINVAL;
  if (pb->stage < 3) FAIL(pb, ASDG_ESTATE, "no bound factor storage");
  const char* src;
  size_t nbytes;
  if (sub < 0) {
    if (!pb->has_coarse) FAIL(pb, ASDG_ESTATE, "no coarse level");
    src = pb->buf[2] + pb->o2.ctiles;
    nbytes = (size_t)pb->n_ctiles * TILE * TILE * 8;
  } else {
    if (sub >= pb->A.n_sub) FAIL(pb, ASDG_EINVAL, "subdomain out of range");
    const SubDesc& d = pb->subs[sub];
    const size_t w = pb->f32 ? 4 : 8;
    if (pb->small) {
      src = pb->buf[1] + pb->o1.tiles + (size_t)d.tile0 * w;
      nbytes = (size_t)d.n * d.n * w;
    } else {
      src = pb->buf[1] + pb->o1.tiles + (size_t)d.tile0 * pb->tile * pb->tile * w;
      nbytes = (size_t)d.nb * (d.nb + 1) / 2 * pb->tile * pb->tile * w;
    }
  }
  if (out_bytes < nbytes) FAIL(pb, ASDG_ENOMEM, "output too small");
  HIPCHK(pb, hipDeviceSynchronize());
  HIPCHK(pb, hipMemcpy(out, src, nbytes, hipMemcpyDeviceToHost));
  return ASDG_OK;
}

asdg_status asdg_export_trace(asdg_problem* pb, int32_t* tasks, uint64_t* times, int64_t max_tasks,
                              int64_t* n_tasks, double* clock_mhz) {
  if (!pb || !n_tasks) return ASDG_EINVAL;
  if (pb->stage < 3) FAIL(pb, ASDG_ESTATE, "nothing traced");
  const int64_t nt = (int64_t)pb->trsv_tasks.size();
  *n_tasks = nt;
  if (clock_mhz) {
    int dev = 0, khz = 0;
    HIPCHK(pb, hipGetDevice(&dev));
    HIPCHK(pb, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *clock_mhz = khz / 1000.0;
  }
  if (!tasks || !times) return ASDG_OK;
  if (max_tasks < nt) FAIL(pb, ASDG_ENOMEM, "output too small");
  std::memcpy(tasks, pb->trsv_tasks.data(), sizeof(int4) * nt);
  HIPCHK(pb, hipDeviceSynchronize());
  HIPCHK(pb, hipMemcpy(times, pb->buf[3] + pb->o3.trace, 3 * 8 * nt, hipMemcpyDeviceToHost));
  return ASDG_OK;
}

int32_t asdg_local_mode(const asdg_problem* pb) {
  if (!pb || pb->stage < 2) return -1;
  return pb->small ? ASDG_LOCAL_SMALL : pb->inv_planned ? ASDG_LOCAL_INVERSE : ASDG_LOCAL_SWEEPS;
}

asdg_status asdg_set_tuning(asdg_problem* pb, int32_t what, int32_t value) {
  if (!pb) return ASDG_EINVAL;
  if (value < 0 || value > 65536) FAIL(pb, ASDG_EINVAL, "tuning value out of range");
  if (what == ASDG_TUNE_CHOL_WG_PER_CU) pb->chol_per_cu = value;
  else if (what == ASDG_TUNE_TRSV_WG_PER_CU) pb->trsv_per_cu = value;
  else if (what == ASDG_TUNE_CHOL_GRID) pb->chol_grid = value;
  else if (what == ASDG_TUNE_TRACE) pb->trace = value;
  else if (what == ASDG_TUNE_LOCAL_INVERSE) pb->local_inverse = value ? 1 : 0;
  else if (what == ASDG_TUNE_SMALL_OFF) pb->small_off = value ? 1 : 0;
  else if (what == ASDG_TUNE_NO_PRECOND) pb->no_precond = value ? 1 : 0;
  else if (what == ASDG_TUNE_INV_WG_PER_CU) pb->inv_per_cu = value;
  else if (what == ASDG_TUNE_HOST_THREADS) pb->host_threads = value;
  else if (what == ASDG_TUNE_FACTOR_SCHEDULE) {
    if (value > 2) FAIL(pb, ASDG_EINVAL, "factorisation schedule: 0 automatic, 1 tile tasks, 2 subdomain tasks");
    pb->factor_sched = value;
  }
  else if (what == ASDG_TUNE_INVERSE_SCHEDULE) {
    if (value > 2) FAIL(pb, ASDG_EINVAL, "inverse-formation schedule: 0 automatic, 1 tile tasks, 2 column tasks");
    pb->inv_sched = value;
  }
  else if (what == ASDG_TUNE_COARSE_PACKED) {
    if (value > 2) FAIL(pb, ASDG_EINVAL, "coarse inverse storage: 0 automatic, 1 packed, 2 dense");
    pb->coarse_packed_mode = value;
  }
  else if (what == ASDG_TUNE_TASK_CHUNK) {
    pb->task_chunk = value;
    if (pb->stage >= 2 && !pb->small) {
      pb->chol_tasks = order_tasks(pb->subs, cholesky_levels, value);
      if (pb->inv_planned) pb->inv_tasks = order_tasks(pb->subs, inverse_levels, value);
      pb->col_tasks = order_col_tasks(pb->subs, value);
      if (pb->stage >= 3) pb->tasks_dirty = true;  // uploaded by the next asdg_factor
    }
  }
  else if (what == ASDG_TUNE_TILE) {
    if (value != 0 && value != 32 && value != 64) FAIL(pb, ASDG_EINVAL, "tile edge: 0 automatic, 32 or 64");
    pb->tile_req = value;  // takes effect at the next asdg_plan
  }
  else if (what == ASDG_TUNE_SYMV_WAVES) {
    if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
      FAIL(pb, ASDG_EINVAL, "waves per work-group of the packed apply must be 1, 2, 4 or 8");
    pb->symv_waves = value;
  } else FAIL(pb, ASDG_EINVAL, "unknown tuning key");
  pb->drop_graph();
  return ASDG_OK;
}

// Autotuner results shared by all handles of the process, keyed by device
// architecture, precision, local-solve representation and size class
// (number of subdomains to a power of two, largest and mean tile rows).
namespace {
std::mutex g_tune_mu;
std::map<std::string, asdg_tune_report> g_tune_cache;

std::string tune_key(const asdg_problem* pb) {
  // tile rows counted in 64-row units whatever the current layout's edge
  double nb_sum = 0.0;
  int nb_max = 0;
  for (const SubDesc& d : pb->subs) {
    const int nb = (d.n + TILE - 1) / TILE;
    nb_sum += nb;
    nb_max = std::max(nb_max, nb);
  }
  const int ns = (int)pb->subs.size();
  int ns_log2 = 0;
  while ((1 << (ns_log2 + 1)) <= ns) ++ns_log2;
  char k[256];
  std::snprintf(k, sizeof(k), "%s|%s|%s|ns2^%d|nbmax%d|nbmean%d", pb->arch.empty() ? "?" : pb->arch.c_str(),
                pb->f32 ? "fp32" : "fp64", pb->inv_planned ? "inverse" : "sweeps", ns_log2, nb_max,
                (int)std::lround(nb_sum / std::max(ns, 1)));
  return k;
}
// Switches the local factors to tiles of edge `tile` inside the bound
// buffers (planned for both edges: tile_search): new task lists, tile
// metadata and subdomain descriptors, uploaded on `s`. The factors must be
// formed again (stage 3).
asdg_status relayout_local(asdg_problem* pb, int tile, hipStream_t s) {
  if (tile == pb->tile) return ASDG_OK;
  if (!pb->tile_search) FAIL(pb, ASDG_ESTATE, "the plan has room for one tile edge only");
  pb->tile = tile;
  plan_local(pb);
  auto up = [&](size_t off, const void* src, size_t nbytes) {
    return nbytes ? hipMemcpyAsync(pb->buf[1] + off, src, nbytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  HIPCHK(pb, up(pb->o1.subs, pb->subs.data(), sizeof(SubDesc) * pb->subs.size()));
  HIPCHK(pb, up(pb->o1.chol, pb->chol_tasks.data(), sizeof(int4) * pb->chol_tasks.size()));
  HIPCHK(pb, up(pb->o1.trsv, pb->trsv_tasks.data(), sizeof(int4) * pb->trsv_tasks.size()));
  HIPCHK(pb, up(pb->o1.meta, pb->tile_meta.data(), sizeof(int4) * pb->tile_meta.size()));
  HIPCHK(pb, up(pb->o1.subt, pb->sub_tasks.data(), sizeof(int4) * pb->sub_tasks.size()));
  HIPCHK(pb, hipStreamSynchronize(s));  // the host lists may change again before the copies complete
  pb->tasks_dirty = false;
  pb->drop_graph();
  if (pb->stage > 3) pb->stage = 3;
  return ASDG_OK;
}
}  // namespace

// Autotuner of the launch shapes and of the local factors' tile edge: every
// candidate is timed on this problem with HIP events on the caller's stream
// (the median of 3 to 15 runs filling about 20 ms; one run when it takes
// more than 20 ms), the fastest is kept. The launch-shape candidates change
// only which work-group does which task, never the arithmetic, so results
// are the same for every choice; the tile edge changes the blocking of the
// factorisation (results equal to rounding).
asdg_status asdg_autotune(asdg_problem* pb, int32_t what, void* stream, asdg_tune_report* rep) {
  if (!pb) return ASDG_EINVAL;
  if ((what & ~(ASDG_AUTOTUNE_FACTOR | ASDG_AUTOTUNE_LOCAL | ASDG_AUTOTUNE_REUSE)) ||
      !(what & (ASDG_AUTOTUNE_FACTOR | ASDG_AUTOTUNE_LOCAL)))
    FAIL(pb, ASDG_EINVAL, "autotune flags: FACTOR and/or LOCAL, optionally REUSE");
  if ((what & ASDG_AUTOTUNE_FACTOR) && pb->stage < 3) FAIL(pb, ASDG_ESTATE, "autotune before asdg_bind");
  if ((what & ASDG_AUTOTUNE_LOCAL) && !(what & ASDG_AUTOTUNE_FACTOR) && pb->stage < 4)
    FAIL(pb, ASDG_ESTATE, "autotune of the local solves before asdg_factor");
  if (pb->solve_open) FAIL(pb, ASDG_ESTATE, "autotune while a solve is in progress");
  hipStream_t s = (hipStream_t)stream;
  asdg_tune_report R;
  std::memset(&R, 0, sizeof(R));
  const std::string key = tune_key(pb);
  if (what & ASDG_AUTOTUNE_REUSE) {
    asdg_tune_report C;
    bool hit = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        C = it->second;
        hit = true;
      }
    }
    if (hit) {
      // the shapes found before for this size class, no timing
      if ((what & ASDG_AUTOTUNE_FACTOR) && pb->tile_search && C.tile != pb->tile) {
        asdg_status e = relayout_local(pb, C.tile, s);
        if (e != ASDG_OK) return e;
      }
      if (what & ASDG_AUTOTUNE_FACTOR) {
        pb->factor_sched = C.factor_schedule;
        pb->inv_sched = C.inverse_schedule;
        pb->chol_per_cu = C.chol_wg_per_cu;
        pb->inv_per_cu = C.inv_wg_per_cu;
        if (C.task_chunk != pb->task_chunk && !pb->small) {
          pb->task_chunk = C.task_chunk;
          pb->chol_tasks = order_tasks(pb->subs, cholesky_levels, C.task_chunk);
          if (pb->inv_planned) pb->inv_tasks = order_tasks(pb->subs, inverse_levels, C.task_chunk);
          pb->col_tasks = order_col_tasks(pb->subs, C.task_chunk);
          pb->tasks_dirty = true;
        }
        asdg_status e = asdg_factor(pb, stream);
        if (e != ASDG_OK) return e;
      }
      if (what & ASDG_AUTOTUNE_LOCAL) {
        pb->trsv_per_cu = C.trsv_wg_per_cu;
        pb->symv_waves = C.symv_waves;
      }
      pb->drop_graph();
      C.candidates = 0;
      C.from_cache = 1;
      C.tile = pb->tile;
      if (rep) *rep = C;
      return ASDG_OK;
    }
  }
  hipEvent_t e0, e1;
  HIPCHK(pb, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    FAIL(pb, ASDG_EHIP, "hipEventCreate failed");
  }
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};

  // one timed factorisation (gather, Cholesky, inverse formation)
  auto time_factor = [&](float& ms) -> asdg_status {
    HIPCHK(pb, hipEventRecord(e0, s));
    asdg_status e = asdg_factor(pb, stream);
    if (e != ASDG_OK) return e;
    HIPCHK(pb, hipEventRecord(e1, s));
    HIPCHK(pb, hipEventSynchronize(e1));
    HIPCHK(pb, hipEventElapsedTime(&ms, e0, e1));
    return ASDG_OK;
  };
  auto tune = [&](int* knob, const std::vector<int>& cand, auto&& run, double& best_ms) -> asdg_status {
    int best = cand.front();
    best_ms = 1e300;
    for (int c : cand) {
      *knob = c;
      float t0 = 0.0f;
      asdg_status e = run(t0);
      if (e != ASDG_OK) return e;
      float m = t0;
      if (t0 < 20.0f) {
        // short runs: the median of an odd number of runs (3 to 15) filling
        // about 20 ms, so that candidates a few percent apart are told apart
        int n = std::max(3, std::min(15, (int)(20.0f / std::max(t0, 1e-3f))));
        if (n % 2 == 0) --n;
        std::vector<float> t(n);
        t[0] = t0;
        for (int k = 1; k < n; ++k)
          if ((e = run(t[k])) != ASDG_OK) return e;
        std::nth_element(t.begin(), t.begin() + n / 2, t.end());
        m = t[n / 2];
      }
      ++R.candidates;
      if (m < best_ms) {
        best_ms = m;
        best = c;
      }
    }
    *knob = best;
    return ASDG_OK;
  };
  // one timed batched local solve (input: zeros permuted into r, which also
  // sets the sweeps' not-yet-written markers)
  double* qz = pb->ptr<double>(3, pb->o3.q);
  DevState* stl = pb->ptr<DevState>(3, pb->o3.st);
  auto time_local = [&](float& ms) -> asdg_status {
    HIPCHK(pb, launch_permute_in(pb->A.np, pb->A.n_cells, pb->ptr<int32_t>(0, pb->o0.perm), qz,
                                 pb->ptr<double>(3, pb->o3.r), nullptr, pb->ptr<void>(3, pb->o3.yl),
                                 pb->ptr<void>(3, pb->o3.zl), pb->f32, nullptr, nullptr, 0.0, 0, s));
    HIPCHK(pb, launch_reset_queues(stl, s));
    HIPCHK(pb, hipEventRecord(e0, s));
    asdg_status e = enqueue_local(pb, s, nullptr);
    if (e != ASDG_OK) return e;
    HIPCHK(pb, hipEventRecord(e1, s));
    HIPCHK(pb, hipEventSynchronize(e1));
    HIPCHK(pb, hipEventElapsedTime(&ms, e0, e1));
    return ASDG_OK;
  };
  if ((what & ASDG_AUTOTUNE_LOCAL) && !pb->small) HIPCHK(pb, hipMemsetAsync(qz, 0, sizeof(double) * pb->n(), s));
  if ((what & ASDG_AUTOTUNE_FACTOR) && (what & ASDG_AUTOTUNE_LOCAL) && pb->tile_search) {
    // the tile edge first (64 or 32 rows; the padding of each subdomain's
    // last tile row against the number of tiles and sweep steps), by the
    // time of one batched local solve, the step repeated every iteration;
    // each edge is factorised once with the default launch shapes
    int tile = pb->tile;
    auto time_tile = [&](float& ms) -> asdg_status {
      if (tile != pb->tile || pb->stage < 4) {
        asdg_status e = relayout_local(pb, tile, s);
        if (e == ASDG_OK) e = asdg_factor(pb, stream);
        if (e != ASDG_OK) return e;
      }
      return time_local(ms);
    };
    double ms = 0.0;
    asdg_status e = tune(&tile, {TILE, 32}, time_tile, ms);
    if (e != ASDG_OK) return e;
    e = relayout_local(pb, tile, s);  // factorised again below with the tuned shapes
    if (e != ASDG_OK) return e;
  }
  if ((what & ASDG_AUTOTUNE_FACTOR) && !pb->small) {
    double ms = 0.0;
    // the schedules first (tile tasks, or one work-group per subdomain / column)
    asdg_status e = tune(&pb->factor_sched, {1, 2}, time_factor, ms);
    if (e != ASDG_OK) return e;
    if (pb->inv_planned) {
      e = tune(&pb->inv_sched, {1, 2}, time_factor, ms);
      if (e != ASDG_OK) return e;
    }
    e = tune(&pb->chol_per_cu, pb->tile == 32 ? std::vector<int>{4, 8} : std::vector<int>{1, 2}, time_factor, ms);
    if (e != ASDG_OK) return e;
    {
      // task order: all subdomains interleaved, or in groups (smaller working set)
      int chunk = pb->task_chunk;
      auto reorder = [&](float& ms1) -> asdg_status {
        pb->chol_tasks = order_tasks(pb->subs, cholesky_levels, chunk);
        if (pb->inv_planned) pb->inv_tasks = order_tasks(pb->subs, inverse_levels, chunk);
        pb->col_tasks = order_col_tasks(pb->subs, chunk);
        pb->tasks_dirty = true;
        return time_factor(ms1);
      };
      std::vector<int> cand{0};
      if (pb->A.n_sub > 64) cand.push_back(64);
      e = tune(&chunk, cand, reorder, ms);
      if (e != ASDG_OK) return e;
      pb->task_chunk = chunk;
      pb->chol_tasks = order_tasks(pb->subs, cholesky_levels, chunk);
      if (pb->inv_planned) pb->inv_tasks = order_tasks(pb->subs, inverse_levels, chunk);
      pb->col_tasks = order_col_tasks(pb->subs, chunk);
      pb->tasks_dirty = true;
    }
    if (pb->inv_planned) {
      e = tune(&pb->inv_per_cu, pb->f32 ? std::vector<int>{1, 2, 3, 4} : std::vector<int>{1, 2}, time_factor, ms);
      if (e != ASDG_OK) return e;
    }
    e = asdg_factor(pb, stream);  // leave the problem factorised with the chosen shapes
    if (e != ASDG_OK) return e;
    R.factor_ms = ms;
  }
  if ((what & ASDG_AUTOTUNE_LOCAL) && !pb->small) {
    double ms = 0.0;
    asdg_status e = pb->inv_planned ? tune(&pb->symv_waves, {1, 2, 4, 8}, time_local, ms)
                                    : tune(&pb->trsv_per_cu, {1, 2, 3, 4}, time_local, ms);
    if (e != ASDG_OK) return e;
    DevState h;
    e = read_state(pb, s, h);
    if (e != ASDG_OK) return e;
    if (h.abort) FAIL(pb, ASDG_EHIP, "local solve wait budget exhausted during autotuning");
    R.local_ms = ms;
  }
  R.chol_wg_per_cu = pb->chol_per_cu > 0 ? pb->chol_per_cu : chol_occupancy(pb->tile);
  R.tile = pb->tile;
  R.inv_wg_per_cu = pb->inv_per_cu > 0 ? pb->inv_per_cu : (pb->f32 ? 4 : 2);
  R.trsv_wg_per_cu = pb->trsv_per_cu > 0 ? pb->trsv_per_cu : 2;
  R.symv_waves = pb->symv_waves > 0 ? pb->symv_waves : 4;
  R.task_chunk = pb->task_chunk;
  R.factor_schedule = pb->small ? 0 : factor_schedule(pb);
  R.inverse_schedule = pb->small || !pb->inv_planned ? 0 : inverse_schedule(pb);
  pb->drop_graph();
  if ((what & (ASDG_AUTOTUNE_FACTOR | ASDG_AUTOTUNE_LOCAL)) == (ASDG_AUTOTUNE_FACTOR | ASDG_AUTOTUNE_LOCAL) && !pb->small) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = R;
  }
  if (rep) *rep = R;
  return ASDG_OK;
}

asdg_status asdg_tune_cache_save(const char* path) {
  if (!path) return ASDG_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return ASDG_EINVAL;
  for (const auto& kv : g_tune_cache) {
    const asdg_tune_report& R = kv.second;
    std::fprintf(f, "%s %d %d %d %d %d %.6f %.6f %d %d %d\n", kv.first.c_str(), R.chol_wg_per_cu, R.inv_wg_per_cu,
                 R.trsv_wg_per_cu, R.symv_waves, R.task_chunk, R.factor_ms, R.local_ms, R.factor_schedule,
                 R.inverse_schedule, R.tile);
  }
  return std::fclose(f) == 0 ? ASDG_OK : ASDG_EINVAL;
}

asdg_status asdg_tune_cache_load(const char* path, int32_t* n_entries) {
  if (!path) return ASDG_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return ASDG_EINVAL;
  std::map<std::string, asdg_tune_report> add;
  char key[256];
  char line[512];
  asdg_tune_report R;
  bool ok = true;
  // one entry per line; the two schedules and the tile edge (last fields)
  // may be missing in files written before they existed (then: automatic,
  // and 64-row tiles)
  while (std::fgets(line, sizeof(line), f)) {
    std::memset(&R, 0, sizeof(R));
    R.tile = TILE;
    const int got = std::sscanf(line, "%255s %d %d %d %d %d %lf %lf %d %d %d", key, &R.chol_wg_per_cu,
                                &R.inv_wg_per_cu, &R.trsv_wg_per_cu, &R.symv_waves, &R.task_chunk, &R.factor_ms,
                                &R.local_ms, &R.factor_schedule, &R.inverse_schedule, &R.tile);
    if (got <= 0) continue;  // blank line
    const bool waves_ok = R.symv_waves == 1 || R.symv_waves == 2 || R.symv_waves == 4 || R.symv_waves == 8;
    if (got < 8 || !waves_ok || R.chol_wg_per_cu < 1 || R.chol_wg_per_cu > 64 || R.inv_wg_per_cu < 1 ||
        R.inv_wg_per_cu > 64 || R.trsv_wg_per_cu < 1 || R.trsv_wg_per_cu > 64 || R.task_chunk < 0 ||
        R.factor_schedule < 0 || R.factor_schedule > 2 || R.inverse_schedule < 0 || R.inverse_schedule > 2 ||
        (R.tile != 32 && R.tile != TILE)) {
      ok = false;
      break;
    }
    add[key] = R;
  }
  std::fclose(f);
  if (!ok) return ASDG_EINVAL;  // nothing is taken from a malformed file
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : add) g_tune_cache[kv.first] = kv.second;
  if (n_entries) *n_entries = (int32_t)add.size();
  return ASDG_OK;
}

}  // extern "C"
