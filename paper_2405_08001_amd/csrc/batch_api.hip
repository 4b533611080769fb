// C ABI of the batched form (declared in include/pncg.h): construction from
// concatenated scenes, steps (single launches or a captured graph of several
// steps), per-scene statistics, and the workgroup-size autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/pncg.h"
#include "batch.h"
#include "host_mesh.h"

using namespace pncg;

namespace {
thread_local std::string g_batch_create_error;
}

namespace {
constexpr int kDefaultPolls = 1 << 21;
constexpr int kNBlocks = 3;
constexpr int kBlocks[kNBlocks] = {256, 512, 1024};
}  // namespace

struct pncg_batch {
  int device = 0, precision = PNCG_FP64;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int nScenes = 0, nV = 0, nT = 0, nWaves = 0;
  std::vector<int> vert_off, tet_off;
  std::vector<void*> allocs;
  int *d_vert_off = nullptr, *d_tet_off = nullptr, *d_wave_off = nullptr;
  std::vector<int> order;   // scenes by decreasing cost
  std::vector<double> cost; // scheduling cost of each scene: its tet count
  // schedule (teams of workgroups, see BatchArgs)
  int nb_cap = 0;           // largest persistent grid over the configurations
  int *d_blk_team = nullptr, *d_blk_rank = nullptr, *d_team_size = nullptr, *d_team_off = nullptr,
      *d_team_scene = nullptr, *d_bar = nullptr;
  double* d_tpart = nullptr;
  int max_team = 1;         // workgroups one scene may use (needs LDS staging when > 1)
  int sched_grid = 0, sched_team = 0, n_teams = 0;
  bool split = false;       // the current schedule has a team of more than one workgroup
  int spin_limit = kDefaultPolls;  // polls before a team barrier gives up
  void* d_elem = nullptr;
  std::vector<char> elem_host;        // host copy of the element records
  std::vector<double> vol_mu, vol_lam;  // V mu and V lam per tet
  int model = PNCG_MODEL_NH;
  int *d_inc = nullptr, *d_inc_vert = nullptr;
  double* d_mass = nullptr;
  uint8_t* d_vflag = nullptr;
  double* d_planes = nullptr;
  double4 *d_x = nullptr, *d_xt = nullptr, *d_xstart = nullptr;
  void *d_g = nullptr, *d_pg = nullptr, *d_p = nullptr;
  int *d_iters = nullptr, *d_reason = nullptr, *d_err = nullptr;
  long long* d_iters_total = nullptr;
  double *d_xa = nullptr, *d_va = nullptr;   // ping-pong state for multi-step runs
  double dhat = 1e-3, kappa = 1e4, eps = 1e-3;
  int iter_max = 100, term = PNCG_TERM_DELTA_E;
  double grav[3] = {0.0, 0.0, -9.8};
  unsigned flags = 0;
  int block = 512, grid = 1, max_grid[kNBlocks] = {1, 1, 1}, max_grid_lds[kNBlocks] = {0, 0, 0};
  int vcap = 0;             // largest scene's vertex count
  bool lds = false;         // stage positions and directions of a scene in LDS
  bool lds_ok = false;      // the largest scene fits in one workgroup's LDS
  // captured multi-step graph
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  const void* g_x = nullptr;
  const void* g_v = nullptr;
  double g_h = 0.0;
  int g_steps = 0, g_block = 0;
  bool g_lds = false;
  int g_team = 0;
};

namespace {

int bfail(pncg_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

#define BCHK(b, call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return bfail(b, PNCG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int balloc(pncg_batch* b, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(n * sizeof(T), 16));
  if (e != hipSuccess) return bfail(b, PNCG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  b->allocs.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return PNCG_OK;
}

template <typename R>
BatchArgs<R> batch_args(pncg_batch* b, double h) {
  BatchArgs<R> A{};
  A.nScenes = b->nScenes;
  A.vcap = b->vcap;
  A.blk_team = b->d_blk_team;
  A.blk_rank = b->d_blk_rank;
  A.team_size = b->d_team_size;
  A.team_off = b->d_team_off;
  A.team_scene = b->d_team_scene;
  A.bar = b->d_bar;
  A.tpart = b->d_tpart;
  A.spin_limit = b->spin_limit;
  A.vert_off = b->d_vert_off;
  A.tet_off = b->d_tet_off;
  A.wave_off = b->d_wave_off;
  A.elem = reinterpret_cast<const ElemRec<R>*>(b->d_elem);
  A.inc = b->d_inc;
  A.inc_vert = b->d_inc_vert;
  A.mass = b->d_mass;
  A.vflag = b->d_vflag;
  A.planes = b->d_planes;
  A.x = b->d_x;
  A.xt = b->d_xt;
  A.xstart = b->d_xstart;
  A.g = reinterpret_cast<R4<R>*>(b->d_g);
  A.pg = reinterpret_cast<R4<R>*>(b->d_pg);
  A.p = reinterpret_cast<R4<R>*>(b->d_p);
  A.dhat = b->dhat;
  A.kappa = b->kappa;
  A.h = h;
  A.h2 = h * h;
  A.eps = b->eps;
  A.grav = mk3(b->grav[0], b->grav[1], b->grav[2]);
  A.iter_max = b->iter_max;
  A.term = b->term;
  A.flags = b->flags;
  A.model = kernel_model(b->model);
  A.iters = b->d_iters;
  A.reason = b->d_reason;
  A.iters_total = b->d_iters_total;
  A.err = b->d_err;
  return A;
}

int block_index(int block) {
  for (int i = 0; i < kNBlocks; ++i)
    if (kBlocks[i] == block) return i;
  return kNBlocks - 1;
}

int grid_for(const pncg_batch* b) {
  const int bi = block_index(b->block);
  return std::max(1, b->lds ? b->max_grid_lds[bi] : b->max_grid[bi]);
}

// Deal the scenes out over teams of workgroups for the current block size
// and staging mode.  Scenes larger than the mean load per workgroup get a
// team of about (tets / mean) workgroups (at most max_team, all with the same
// blockIdx % 8, which the dispatcher places on one XCD); the rest go to
// single workgroups, and every remaining scene joins the least loaded team
// (longest first).  Uploaded on the stream, which is then synchronised; not
// called while a graph is being captured.
int ensure_schedule(pncg_batch* b) {
  const int NB = grid_for(b);
  const int maxG = b->lds ? std::min(b->max_team, kMaxTeam) : 1;
  if (NB == b->sched_grid && maxG == b->sched_team) return PNCG_OK;
  const std::vector<double>& cost = b->cost;
  double total = 0.0;
  for (double c : cost) total += c;
  const double avg = total / NB;
  std::vector<std::vector<int>> pool(kXcds);
  for (int q = NB - 1; q >= 0; --q) pool[q % kXcds].push_back(q);   // back() = lowest free index
  struct TeamB { std::vector<int> blocks, scenes; double load; };
  std::vector<TeamB> teams;
  size_t i = 0;
  for (; i < b->order.size() && maxG > 1; ++i) {
    const int s = b->order[i];
    int G = std::min(maxG, (int)(cost[s] / avg + 0.5));
    if (G < 2) break;
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (pool[y].size() > pool[x].size()) x = y;
    G = std::min<int>(G, (int)pool[x].size());
    if (G < 2) break;
    TeamB t{{}, {s}, cost[s] / G};
    for (int k = 0; k < G; ++k) { t.blocks.push_back(pool[x].back()); pool[x].pop_back(); }
    teams.push_back(t);
  }
  for (int x = 0; x < kXcds; ++x)
    for (int q : pool[x]) teams.push_back(TeamB{{q}, {}, 0.0});
  for (; i < b->order.size(); ++i) {
    const int s = b->order[i];
    size_t best = 0;
    for (size_t t = 1; t < teams.size(); ++t)
      if (teams[t].load < teams[best].load) best = t;
    teams[best].scenes.push_back(s);
    teams[best].load += cost[s] / teams[best].blocks.size();
  }
  std::vector<int> blk_team(NB, 0), blk_rank(NB, 0), tsize, toff(1, 0), tscene;
  bool split = false;
  for (size_t t = 0; t < teams.size(); ++t) {
    for (size_t k = 0; k < teams[t].blocks.size(); ++k) {
      blk_team[teams[t].blocks[k]] = (int)t;
      blk_rank[teams[t].blocks[k]] = (int)k;
    }
    tsize.push_back((int)teams[t].blocks.size());
    split |= teams[t].blocks.size() > 1;
    tscene.insert(tscene.end(), teams[t].scenes.begin(), teams[t].scenes.end());
    toff.push_back((int)tscene.size());
  }
  BCHK(b, hipMemcpyAsync(b->d_blk_team, blk_team.data(), sizeof(int) * NB, hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->d_blk_rank, blk_rank.data(), sizeof(int) * NB, hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->d_team_size, tsize.data(), sizeof(int) * tsize.size(), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->d_team_off, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->d_team_scene, tscene.data(), sizeof(int) * tscene.size(), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  b->sched_grid = NB;
  b->sched_team = maxG;
  b->n_teams = (int)teams.size();
  b->split = split;
  return PNCG_OK;
}

void launch(pncg_batch* b, double h, const double* x, const double* v, double* xo, double* vo) {
  const int grid = b->sched_grid;
  if (b->split) launch_team_reset(b->d_bar, b->n_teams, b->stream);
  if (b->precision == PNCG_MIXED)
    launch_batch_step<float>(batch_args<float>(b, h), b->block, grid, b->lds, x, v, xo, vo, b->stream);
  else
    launch_batch_step<double>(batch_args<double>(b, h), b->block, grid, b->lds, x, v, xo, vo, b->stream);
}

int check_err(pncg_batch* b) {
  int e = 0;
  BCHK(b, hipMemcpyAsync(&e, b->d_err, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  if (e & kErrInverted) return bfail(b, PNCG_E_INVERTED, inverted_message(b->model));
  if (e & kErrPenetration) return bfail(b, PNCG_E_PENETRATION, "a vertex is on or behind its plane");
  if (e & kErrTeam)
    return bfail(b, PNCG_E_HIP, "a team barrier timed out (the workgroups of a team were not all resident); "
                                "results are invalid: call pncg_batch_set_split(b, 1)");
  return PNCG_OK;
}

template <typename R>
int upload_elems(pncg_batch* b, const std::vector<int>& tets_g, const std::vector<double>& Bm,
                 const std::vector<double>& vol, const double* E, const double* nu) {
  std::vector<ElemRec<R>> rec(b->nT);
  b->vol_mu.resize(b->nT);
  b->vol_lam.resize(b->nT);
  for (int e = 0; e < b->nT; ++e) {
    for (int a = 0; a < 4; ++a) rec[e].v[a] = tets_g[4 * e + a];
    for (int j = 0; j < 9; ++j) rec[e].B[j] = R(Bm[9 * (size_t)e + j]);
    const double mu = E[e] / (2.0 * (1.0 + nu[e])), lam = E[e] * nu[e] / ((1.0 + nu[e]) * (1.0 - 2.0 * nu[e]));
    b->vol_mu[e] = vol[e] * mu;
    b->vol_lam[e] = vol[e] * lam;
    rec[e].vmu = R(vol[e] * mu);
    rec[e].vlam = R(vol[e] * record_lam(b->model, mu, lam));
  }
  int rc = balloc(b, reinterpret_cast<ElemRec<R>**>(&b->d_elem), (size_t)b->nT);
  if (rc) return rc;
  const char* bytes = reinterpret_cast<const char*>(rec.data());
  b->elem_host.assign(bytes, bytes + sizeof(ElemRec<R>) * (size_t)b->nT);
  BCHK(b, hipMemcpy(b->d_elem, rec.data(), sizeof(ElemRec<R>) * (size_t)b->nT, hipMemcpyHostToDevice));
  return PNCG_OK;
}

// Rewrite the records' lam for the current model and upload them.
template <typename R>
int repack_elems(pncg_batch* b) {
  ElemRec<R>* rec = reinterpret_cast<ElemRec<R>*>(b->elem_host.data());
  for (int e = 0; e < b->nT; ++e) rec[e].vlam = R(record_lam(b->model, b->vol_mu[e], b->vol_lam[e]));
  BCHK(b, hipMemcpy(b->d_elem, rec, sizeof(ElemRec<R>) * (size_t)b->nT, hipMemcpyHostToDevice));
  return PNCG_OK;
}

// Persistent grid size: resident workgroups per CU times the CU count (0 when
// the LDS-staged kernel cannot be resident at all).
int max_active(pncg_batch* b, int block, bool lds, int kmodel, int* out) {
  int n = 0;
  hipDeviceProp_t prop;
  BCHK(b, hipGetDeviceProperties(&prop, b->device));
  if (b->precision == PNCG_MIXED)
    BCHK(b, batch_occupancy<float>(block, lds, b->vcap, kmodel, &n));
  else
    BCHK(b, batch_occupancy<double>(block, lds, b->vcap, kmodel, &n));
  *out = lds ? n * prop.multiProcessorCount : std::max(1, n) * prop.multiProcessorCount;
  return PNCG_OK;
}

// Persistent grid sizes of every block size, with and without LDS staging,
// for kernel model kmodel; lds_ok: the staged kernel is resident at all.
int size_grids(pncg_batch* b, int kmodel, int* grid, int* grid_lds, bool* lds_ok) {
  int rc;
  for (int i = 0; i < kNBlocks; ++i)
    if ((rc = max_active(b, kBlocks[i], false, kmodel, &grid[i]))) return rc;
  *lds_ok = false;
  for (int i = 0; i < kNBlocks; ++i) grid_lds[i] = 0;
  hipDeviceProp_t prop;
  BCHK(b, hipGetDeviceProperties(&prop, b->device));
  const size_t need = b->precision == PNCG_MIXED ? batch_lds_bytes<float>(b->vcap) : batch_lds_bytes<double>(b->vcap);
  // static LDS of the kernel is 8 doubles per wave: at most 1 KiB
  if (need + 1024 <= prop.sharedMemPerBlock) {
    *lds_ok = true;
    for (int i = 0; i < kNBlocks; ++i) {
      if ((rc = max_active(b, kBlocks[i], true, kmodel, &grid_lds[i]))) return rc;
      if (grid_lds[i] < 1) *lds_ok = false;
    }
  }
  return PNCG_OK;
}

void drop_graph(pncg_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_steps = 0;
}

}  // namespace

extern "C" {

int pncg_batch_create(pncg_batch** out, const pncg_opts* o, int32_t nScenes, const int32_t* vert_off,
                      const double* X, const int32_t* tet_off, const int32_t* tets, const int32_t* tri_off,
                      const int32_t* tris, const double* E, const double* nu, const double* rho,
                      const double* planes) {
  if (!out) {
    g_batch_create_error = "out is NULL";
    return PNCG_E_INVAL;
  }
  *out = nullptr;
  auto fail_create = [](int code, const std::string& m) {
    g_batch_create_error = m;
    return code;
  };
  if (nScenes <= 0 || !vert_off || !X || !tet_off || !tets || !tri_off || !E || !nu || !rho)
    return fail_create(PNCG_E_INVAL, "bad batch arguments");
  const int precision = o ? o->precision : PNCG_FP64;
  if (precision != PNCG_FP64 && precision != PNCG_MIXED) return fail_create(PNCG_E_INVAL, "bad precision");
  if (vert_off[0] != 0 || tet_off[0] != 0 || tri_off[0] != 0) return fail_create(PNCG_E_INVAL, "offsets must start at 0");
  for (int s = 0; s < nScenes; ++s)
    if (vert_off[s + 1] <= vert_off[s] || tet_off[s + 1] <= tet_off[s] || tri_off[s + 1] < tri_off[s])
      return fail_create(PNCG_E_INVAL, "offsets must increase (every scene needs vertices and tets)");
  const int nV = vert_off[nScenes], nT = tet_off[nScenes];
  for (long long i = 0; i < 3LL * nV; ++i)
    if (!std::isfinite(X[i])) return fail_create(PNCG_E_NONFINITE, "non-finite rest position");
  for (int e = 0; e < nT; ++e)
    if (!(E[e] > 0.0) || !(nu[e] >= 0.0 && nu[e] < 0.5) || !(rho[e] > 0.0) || !std::isfinite(E[e]) ||
        !std::isfinite(rho[e]))
      return fail_create(PNCG_E_INVAL, "material out of range");
  std::vector<int> tets_g(4 * (size_t)nT);
  std::vector<uint8_t> fl(nV, 0);
  std::vector<int> inc, incv, wave_off(nScenes + 1, 0);
  std::vector<double> Bm, vol, mass(nV, 0.0);
  Bm.reserve(9 * (size_t)nT);
  vol.reserve(nT);
  for (int s = 0; s < nScenes; ++s) {
    const int sv = vert_off[s + 1] - vert_off[s], st = tet_off[s + 1] - tet_off[s];
    const int* lt = tets + 4 * (size_t)tet_off[s];
    for (long long i = 0; i < 4LL * st; ++i)
      if (lt[i] < 0 || lt[i] >= sv) return fail_create(PNCG_E_INVAL, "tet index out of range in scene " + std::to_string(s));
    std::vector<double> b_s, v_s;
    const int bad = rest_shape(X + 3 * (size_t)vert_off[s], lt, st, b_s, v_s);
    if (bad >= 0) return fail_create(PNCG_E_INVERTED, "rest tet with det <= 0 in scene " + std::to_string(s));
    Bm.insert(Bm.end(), b_s.begin(), b_s.end());
    vol.insert(vol.end(), v_s.begin(), v_s.end());
    for (long long i = 0; i < 4LL * st; ++i) tets_g[4 * (size_t)tet_off[s] + i] = lt[i] + vert_off[s];
    if (!pack_incidence(sv, lt, st, vert_off[s], inc, incv, tet_off[s]))
      return fail_create(PNCG_E_INVAL, "a vertex belongs to more than 64 tets");
    wave_off[s + 1] = (int)(inc.size() / kWave);
    for (int t = tri_off[s]; t < tri_off[s + 1]; ++t)
      for (int j = 0; j < 3; ++j) {
        const int v = tris[3 * (size_t)t + j];
        if (v < 0 || v >= sv) return fail_create(PNCG_E_INVAL, "triangle index out of range");
        fl[v + vert_off[s]] |= kSurface;
      }
  }
  for (int e = 0; e < nT; ++e)
    for (int a = 0; a < 4; ++a) mass[tets_g[4 * (size_t)e + a]] += rho[e] * vol[e] / 4.0;
  std::vector<double> pl(4 * (size_t)nScenes, 0.0);
  if (planes) {
    for (int s = 0; s < nScenes; ++s) {
      const double* q = planes + 4 * s;
      const double n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
      if (n2 != 0.0 && std::fabs(std::sqrt(n2) - 1.0) > 1e-6) return fail_create(PNCG_E_INVAL, "plane normal must be unit or zero");
      for (int j = 0; j < 4; ++j) pl[4 * s + j] = q[j];
    }
  }
  // scenes by decreasing size (scheduling order)
  std::vector<int> order(nScenes);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return tet_off[a + 1] - tet_off[a] > tet_off[c + 1] - tet_off[c];
  });

  pncg_batch* b = new pncg_batch();
  b->device = o ? o->device : 0;
  b->precision = precision;
  b->stream = o ? reinterpret_cast<hipStream_t>(o->stream) : nullptr;
  b->nScenes = nScenes;
  b->nV = nV;
  b->nT = nT;
  b->nWaves = (int)(inc.size() / kWave);
  b->vert_off.assign(vert_off, vert_off + nScenes + 1);
  b->order = order;
  for (int s = 0; s < nScenes; ++s) b->cost.push_back(double(tet_off[s + 1] - tet_off[s]));
  for (int s = 0; s < nScenes; ++s) b->vcap = std::max(b->vcap, vert_off[s + 1] - vert_off[s]);
  b->tet_off.assign(tet_off, tet_off + nScenes + 1);
  int rc = PNCG_OK;
  auto fin = [&](int code) {
    if (code != PNCG_OK) {
      g_batch_create_error = b->err;
      pncg_batch_destroy(b);
      return code;
    }
    *out = b;
    return PNCG_OK;
  };
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= b->device) return fin(bfail(b, PNCG_E_HIP, "no HIP device"));
  if (hipSetDevice(b->device) != hipSuccess) return fin(bfail(b, PNCG_E_HIP, "hipSetDevice failed"));
  if (!b->stream) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return fin(bfail(b, PNCG_E_HIP, "stream creation failed"));
    b->own_stream = true;
  }
  const size_t r4 = precision == PNCG_MIXED ? sizeof(float4) : sizeof(double4);
  if ((rc = balloc(b, &b->d_vert_off, nScenes + 1)) ||
      (rc = balloc(b, &b->d_tet_off, nScenes + 1)) || (rc = balloc(b, &b->d_wave_off, nScenes + 1)) ||
      (rc = balloc(b, &b->d_inc, inc.size())) || (rc = balloc(b, &b->d_inc_vert, incv.size())) ||
      (rc = balloc(b, &b->d_mass, nV)) || (rc = balloc(b, &b->d_vflag, nV)) ||
      (rc = balloc(b, &b->d_planes, 4 * (size_t)nScenes)) || (rc = balloc(b, &b->d_x, nV)) ||
      (rc = balloc(b, &b->d_xt, nV)) || (rc = balloc(b, &b->d_xstart, nV)) ||
      (rc = balloc(b, (char**)&b->d_g, r4 * nV)) || (rc = balloc(b, (char**)&b->d_pg, r4 * nV)) ||
      (rc = balloc(b, (char**)&b->d_p, r4 * nV)) || (rc = balloc(b, &b->d_iters, nScenes)) ||
      (rc = balloc(b, &b->d_reason, nScenes)) || (rc = balloc(b, &b->d_err, 1)) ||
      (rc = balloc(b, &b->d_iters_total, nScenes)) || (rc = balloc(b, &b->d_xa, 3 * (size_t)nV)) ||
      (rc = balloc(b, &b->d_va, 3 * (size_t)nV)))
    return fin(rc);
  rc = precision == PNCG_MIXED ? upload_elems<float>(b, tets_g, Bm, vol, E, nu)
                               : upload_elems<double>(b, tets_g, Bm, vol, E, nu);
  if (rc) return fin(rc);
#define UP(dst, src, n)                                                                          \
  if (hipMemcpy(dst, src, n, hipMemcpyHostToDevice) != hipSuccess) return fin(bfail(b, PNCG_E_HIP, "upload failed"));
  UP(b->d_vert_off, vert_off, sizeof(int) * (nScenes + 1));
  UP(b->d_tet_off, tet_off, sizeof(int) * (nScenes + 1));
  UP(b->d_wave_off, wave_off.data(), sizeof(int) * (nScenes + 1));
  UP(b->d_inc, inc.data(), sizeof(int) * inc.size());
  UP(b->d_inc_vert, incv.data(), sizeof(int) * incv.size());
  UP(b->d_mass, mass.data(), sizeof(double) * nV);
  UP(b->d_vflag, fl.data(), nV);
  UP(b->d_planes, pl.data(), sizeof(double) * pl.size());
#undef UP
  if (hipMemset(b->d_iters_total, 0, sizeof(long long) * nScenes) != hipSuccess ||
      hipMemset(b->d_err, 0, sizeof(int)) != hipSuccess)
    return fin(bfail(b, PNCG_E_HIP, "memset failed"));
  // the schedule buffers hold the largest grid of any model
  for (int km = 0; km < 3; ++km) {
    int g[kNBlocks], gl[kNBlocks];
    bool ok;
    if ((rc = size_grids(b, km, g, gl, &ok))) return fin(rc);
    for (int i = 0; i < kNBlocks; ++i) b->nb_cap = std::max({b->nb_cap, g[i], gl[i]});
  }
  if ((rc = size_grids(b, kernel_model(b->model), b->max_grid, b->max_grid_lds, &b->lds_ok))) return fin(rc);
  b->lds = b->lds_ok;
  b->max_team = b->lds ? kMaxTeam : 1;
  if ((rc = balloc(b, &b->d_blk_team, b->nb_cap)) || (rc = balloc(b, &b->d_blk_rank, b->nb_cap)) ||
      (rc = balloc(b, &b->d_team_size, b->nb_cap)) || (rc = balloc(b, &b->d_team_off, b->nb_cap + 1)) ||
      (rc = balloc(b, &b->d_team_scene, nScenes)) || (rc = balloc(b, &b->d_bar, b->nb_cap)) ||
      (rc = balloc(b, &b->d_tpart, (size_t)b->nb_cap * 2 * kMaxTeam * 8)))
    return fin(rc);
  return fin(ensure_schedule(b));
}

void pncg_batch_destroy(pncg_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

const char* pncg_batch_last_error(const pncg_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

int pncg_batch_set_params(pncg_batch* b, double dhat, double kappa, int32_t iter_max, double eps, int32_t term,
                          const double* gravity, uint32_t flags) {
  if (!b) return PNCG_E_INVAL;
  if (!(dhat > 0.0) || !(kappa >= 0.0) || iter_max < 1 || !(eps >= 0.0) || (term < 0 || term > 2) ||
      (flags & ~(3u | PNCG_BETA_MASK)) || (flags & PNCG_BETA_MASK) > PNCG_BETA_HZ)
    return bfail(b, PNCG_E_INVAL, "bad batch parameters");
  b->dhat = dhat;
  b->kappa = kappa;
  b->iter_max = iter_max;
  b->eps = eps;
  b->term = term;
  if (gravity) std::memcpy(b->grav, gravity, sizeof(b->grav));
  b->flags = flags;
  drop_graph(b);
  return PNCG_OK;
}

int pncg_batch_set_block(pncg_batch* b, int32_t block) {
  if (!b) return PNCG_E_INVAL;
  if (block != 256 && block != 512 && block != 1024) return bfail(b, PNCG_E_INVAL, "block must be 256, 512 or 1024");
  b->block = block;
  drop_graph(b);
  return ensure_schedule(b);
}

int pncg_batch_set_model(pncg_batch* b, int32_t model) {
  if (!b) return PNCG_E_INVAL;
  if (model < PNCG_MODEL_NH || model > PNCG_MODEL_FCR) return bfail(b, PNCG_E_INVAL, "unknown material model");
  BCHK(b, hipSetDevice(b->device));
  if (b->stream) BCHK(b, hipStreamSynchronize(b->stream));
  b->model = model;
  int rc = b->precision == PNCG_MIXED ? repack_elems<float>(b) : repack_elems<double>(b);
  if (rc) return rc;
  if ((rc = size_grids(b, kernel_model(model), b->max_grid, b->max_grid_lds, &b->lds_ok))) return rc;
  if (!b->lds_ok) {
    b->lds = false;
    b->max_team = 1;
  }
  drop_graph(b);
  b->sched_grid = 0;
  return ensure_schedule(b);
}

int pncg_batch_set_staging(pncg_batch* b, int32_t lds) {
  if (!b) return PNCG_E_INVAL;
  if (lds != 0 && lds != 1) return bfail(b, PNCG_E_INVAL, "staging must be 0 or 1");
  if (lds && !b->lds_ok) return bfail(b, PNCG_E_INVAL, "the largest scene does not fit in one workgroup's LDS");
  b->lds = lds != 0;
  drop_graph(b);
  return ensure_schedule(b);
}

int pncg_batch_set_split(pncg_batch* b, int32_t max_team, int32_t max_polls) {
  if (!b) return PNCG_E_INVAL;
  if (max_team < 1 || max_team > kMaxTeam) return bfail(b, PNCG_E_INVAL, "max_team must be in [1, 8]");
  if (max_polls < 0) return bfail(b, PNCG_E_INVAL, "max_polls must be >= 0");
  b->max_team = max_team;
  b->spin_limit = max_polls ? max_polls : kDefaultPolls;
  drop_graph(b);
  return ensure_schedule(b);
}

int pncg_batch_get_config(pncg_batch* b, int32_t* block, int32_t* lds, int32_t* max_team, int32_t* teams) {
  if (!b) return PNCG_E_INVAL;
  if (block) *block = b->block;
  if (lds) *lds = b->lds ? 1 : 0;
  if (max_team) *max_team = b->max_team;
  if (teams) *teams = b->n_teams;
  return PNCG_OK;
}

int pncg_batch_step(pncg_batch* b, const double* x, const double* v, double h, double* x_out, double* v_out) {
  if (!b || !x || !v || !x_out || !v_out) return bfail(b, PNCG_E_INVAL, "NULL argument");
  if (!(h > 0.0) || !std::isfinite(h)) return bfail(b, PNCG_E_INVAL, "need a finite h > 0");
  BCHK(b, hipSetDevice(b->device));
  int rc = ensure_schedule(b);
  if (rc) return rc;
  BCHK(b, hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
  launch(b, h, x, v, x_out, v_out);
  BCHK(b, hipGetLastError());
  return check_err(b);
}

int pncg_batch_run(pncg_batch* b, double* x, double* v, double h, int32_t nsteps) {
  if (!b || !x || !v || nsteps < 1) return bfail(b, PNCG_E_INVAL, "bad arguments");
  if (!(h > 0.0) || !std::isfinite(h)) return bfail(b, PNCG_E_INVAL, "need a finite h > 0");
  BCHK(b, hipSetDevice(b->device));
  int rc = ensure_schedule(b);
  if (rc) return rc;
  if (!b->gexec || b->g_x != x || b->g_v != v || b->g_h != h || b->g_steps != nsteps || b->g_block != b->block ||
      b->g_lds != b->lds || b->g_team != b->max_team) {
    drop_graph(b);
    BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const size_t n3 = 3 * (size_t)b->nV;
    double *xa = x, *va = v, *xb = b->d_xa, *vb = b->d_va;
    for (int i = 0; i < nsteps; ++i) {
      launch(b, h, xa, va, xb, vb);
      std::swap(xa, xb);
      std::swap(va, vb);
    }
    if (xa != x) {
      (void)hipMemcpyAsync(x, xa, sizeof(double) * n3, hipMemcpyDeviceToDevice, b->stream);
      (void)hipMemcpyAsync(v, va, sizeof(double) * n3, hipMemcpyDeviceToDevice, b->stream);
    }
    hipError_t e = hipStreamEndCapture(b->stream, &b->graph);
    if (e != hipSuccess) return bfail(b, PNCG_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    BCHK(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->g_x = x;
    b->g_v = v;
    b->g_h = h;
    b->g_steps = nsteps;
    b->g_block = b->block;
    b->g_lds = b->lds;
    b->g_team = b->max_team;
  }
  BCHK(b, hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));  // outside the graph
  BCHK(b, hipGraphLaunch(b->gexec, b->stream));
  return check_err(b);
}

int pncg_batch_stats(pncg_batch* b, int32_t* iters, int32_t* reason, int64_t* iters_total) {
  if (!b) return PNCG_E_INVAL;
  BCHK(b, hipSetDevice(b->device));
  if (iters) BCHK(b, hipMemcpyAsync(iters, b->d_iters, sizeof(int) * b->nScenes, hipMemcpyDeviceToHost, b->stream));
  if (reason) BCHK(b, hipMemcpyAsync(reason, b->d_reason, sizeof(int) * b->nScenes, hipMemcpyDeviceToHost, b->stream));
  if (iters_total)
    BCHK(b, hipMemcpyAsync(iters_total, b->d_iters_total, sizeof(long long) * b->nScenes, hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  return PNCG_OK;
}

int pncg_batch_autotune(pncg_batch* b, const double* x, const double* v, double h, int32_t reps, int32_t* block_out) {
  if (!b || !x || !v || reps < 1) return bfail(b, PNCG_E_INVAL, "bad arguments");
  BCHK(b, hipSetDevice(b->device));
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  BCHK(b, hipEventCreate(&e1));
  float best = 1e30f;
  int best_b = b->block, best_t = b->max_team;
  bool best_l = b->lds;
  // (staging, max team): device memory; LDS; LDS with large scenes split
  // over up to 2 or up to 8 workgroups
  const int modes[4][2] = {{0, 1}, {1, 1}, {1, 2}, {1, kMaxTeam}};
  for (int m = 0; m < (b->lds_ok ? 4 : 1); ++m)
    for (int i = 0; i < kNBlocks; ++i) {
      b->block = kBlocks[i];
      b->lds = modes[m][0] == 1;
      b->max_team = modes[m][1];
      int rc = ensure_schedule(b);
      if (rc) return rc;
      launch(b, h, x, v, b->d_xa, b->d_va);  // warm-up
      BCHK(b, hipEventRecord(e0, b->stream));
      for (int r = 0; r < reps; ++r) launch(b, h, x, v, b->d_xa, b->d_va);
      BCHK(b, hipEventRecord(e1, b->stream));
      BCHK(b, hipEventSynchronize(e1));
      float ms = 0.0f;
      BCHK(b, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_b = kBlocks[i];
        best_l = b->lds;
        best_t = b->max_team;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->block = best_b;
  b->lds = best_l;
  b->max_team = best_t;
  drop_graph(b);
  int rc = ensure_schedule(b);
  if (rc) return rc;
  if (block_out) *block_out = best_b;
  return check_err(b);
}

}  // extern "C"
