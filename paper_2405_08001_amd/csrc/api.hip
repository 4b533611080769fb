// Host runtime and C ABI of libpncg (declared in include/pncg.h).
//
// The context keeps the mesh in the layouts the kernels want: one 64-byte
// (mixed) or 112-byte (float64) record per tet holding its indices, the rows
// of D_m^{-1} and V mu, V lam; positions as padded double4 (one load per
// gathered vertex); per-vertex float32 or float64 vectors as padded 4-vectors;
// and the vertex -> (tet, corner) incidence packed so that no vertex's lanes
// straddle a 64-lane wave.  A time step runs entirely on the device: the host
// launches chunks of iterations and reads a small status block between
// chunks (to stop, or to rebuild the candidate list when the accumulated
// displacement bound exceeds half the skin).
#include <algorithm>
#include <climits>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pncg.h"
#include "adjoint.h"
#include "host_mesh.h"
#include "internal.h"
#include "kernels.h"

using namespace pncg;

namespace {

thread_local std::string g_create_error;

// Reduction scratch of the allocation-free step (pncg_step_dev_noalloc): the
// step status, the per-block partials of the three per-iteration kernels and
// the per-iteration scalar records.  Every call on a device shares that
// device's copy; each call initialises what it reads before reading it.
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr size_t kScratchStatus = 0;                                     // StepStatus
constexpr size_t kScratchPartGrad = 256;                                 // [kMaxGrid][8] doubles
constexpr size_t kScratchPartDir = kScratchPartGrad + 8 * sizeof(double) * kMaxGrid;   // [kMaxGrid][4]
constexpr size_t kScratchPartNarrow = kScratchPartDir + 4 * sizeof(double) * kMaxGrid; // [kMaxGrid]
constexpr size_t kScratchScal = kScratchPartNarrow + sizeof(double) * kMaxGrid;        // IterScal[...]
constexpr int kScratchScalRecords = (int)((kScratchBytes - kScratchScal) / sizeof(IterScal));
static_assert(sizeof(StepStatus) <= kScratchPartGrad, "step status does not fit its scratch slot");
static_assert(kScratchScal % alignof(IterScal) == 0, "misaligned scratch records");
static_assert(kScratchScalRecords - 2 == PNCG_NOALLOC_ITER_MAX, "PNCG_NOALLOC_ITER_MAX does not match the scratch");

// Device address of `scratch` on each device, taken once with that device
// current (the array's host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct pncg_ctx {
  int device = 0;
  int precision = PNCG_FP64;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool dev_ready = false;
  int scatter = PNCG_SCATTER_SEGMENTED;   // resolved PNCG_SCATTER_* of the options
  void* d_static = nullptr;    // this device's `scratch` (pncg_step_dev_noalloc)
  bool noalloc = false;        // inside pncg_step_dev_noalloc: no device allocation allowed
  int chunk = 16;
  bool graphs = true;                      // rebuilds replayed from captured graphs
  long long last_ncand = 0;                // size of the last solver list the host has read
  bool list_valid = false;                 // d_cand / xbuild hold the solver list of the last step
  double last_D_end = 0.0;                 // its displacement bound from the build at that step's end
  struct RebuildGraph {
    hipGraphExec_t exec = nullptr;
    unsigned char key[sizeof(Broad) + sizeof(PairIndex) + 8 * sizeof(void*) + 4 * sizeof(double)] = {};
  } rgraph[2];                             // by the buffer the list is built from (x0, x1)
  std::string err;
  int state = 0;  // 0 created, 1 mesh, 2 material

  // host mesh
  int nV = 0, nT = 0, nF = 0, nE = 0, nSV = 0;
  std::vector<double> X;
  std::vector<int> tets, tris, edges, surf, oid;
  std::vector<double> vol, Bm;  // Bm: [nT][9] rows of D_m^{-1}
  std::vector<double> E, nu, rho, mass;
  std::vector<uint8_t> vflag;
  std::vector<int> inc, inc_vert;
  int nWaves = 0;
  int model = PNCG_MODEL_NH;   // elastic density (PNCG_MODEL_*)

  // contact / solver parameters
  double dhat = 1e-3, kappa = 0.0, cell_user = 0.0, cell = 0.0, skin = 0.0, skin_user = 0.0, lmean = 0.0;
  Planes planes{};
  unsigned cflags = 0;
  int iter_max = 100, term = PNCG_TERM_DELTA_E;
  double eps = 1e-3;
  double grav[3] = {0.0, 0.0, -9.8};
  unsigned sflags = 0;
  std::vector<int> fixed;
  std::vector<double> fixed_target;

  // device memory
  std::vector<void*> allocs;
  void* d_elem = nullptr;
  int* d_inc = nullptr;
  int* d_inc_vert = nullptr;
  double* d_mass = nullptr;
  uint8_t* d_vflag = nullptr;
  double4* d_target = nullptr;
  double4* d_xbuild = nullptr;
  double4 *d_x0 = nullptr, *d_x1 = nullptr, *d_xt = nullptr, *d_xstart = nullptr;
  void *d_g = nullptr, *d_pg = nullptr, *d_p0 = nullptr, *d_p1 = nullptr;
  double* d_acc = nullptr;
  int *d_tris = nullptr, *d_edges = nullptr, *d_surf = nullptr, *d_oid = nullptr;
  unsigned long long *d_excl_pt = nullptr, *d_excl_ee = nullptr;
  int n_excl_pt = 0, n_excl_ee = 0;
  int2* d_cand = nullptr;
  long long cand_cap = 0;
  // segmented scatter: the list's per-vertex entry index and the run
  // partials of its pair terms (sized by cand_cap)
  int *d_vcnt = nullptr, *d_coff = nullptr, *d_cent = nullptr, *d_cent_tmp = nullptr, *d_pl_tmp = nullptr,
      *d_big = nullptr;
  unsigned long long* d_ckey_tmp = nullptr;
  int2 *d_wvert = nullptr, *d_wrange = nullptr;   // per incidence wave: first / last vertex, entry range
  double* d_rp = nullptr;      // [4 cap][6] run partials of the pair entries
  int4* d_pv = nullptr;        // [cap] corner vertices of each pair
  // explicit candidate lists (pncg_set_candidates_override), kind in the pair
  bool ovr_set[2] = {false, false};
  std::vector<int2> ovr[2];
  int2* d_ovr = nullptr;
  long long n_ovr = 0;
  bool ovr_uploaded = false;
  long long* d_ncand = nullptr;
  IterScal* d_scal = nullptr;
  int scal_cap = 0;
  // splitting computation: objects as contiguous vertex / tet ranges
  int nObj = 0, oscal_cap = 0;
  bool split_ready = false;
  int *d_vobj = nullptr, *d_voff = nullptr, *d_toff = nullptr;
  ObjScal* d_oscal = nullptr;
  double *d_vdots = nullptr, *d_tphp = nullptr, *d_vphp = nullptr, *d_opair = nullptr;
  StepStatus* d_status = nullptr;
  StepStatus* h_status = nullptr;  // pinned [2]: the step loop reads one while the other is in flight
  hipEvent_t st_ev[2] = {nullptr, nullptr};  // recorded after each status copy
  long long* h_n = nullptr;        // pinned [2]
  double* d_part_grad = nullptr;
  double* d_part_dir = nullptr;
  double* d_part_narrow = nullptr;
  double* d_io = nullptr;          // [4][nV][3] staging for host inputs/outputs
  double* d_scalar = nullptr;      // [8]
  // broad phase
  int tsize = 0;
  int *d_count = nullptr, *d_start = nullptr;
  double4 *d_item_lo = nullptr, *d_item_hi = nullptr;
  long long *d_item_cnt = nullptr, *d_item_off = nullptr;
  long long ent_cap = 0;
  unsigned long long *d_ent_key = nullptr, *d_bkt_key = nullptr;
  int *d_ent_item = nullptr, *d_bkt_item = nullptr, *d_ent_rank = nullptr;
  double4 *d_bkt_lo = nullptr, *d_bkt_hi = nullptr;
  int4* d_bkt_ids = nullptr;
  long long *d_part_cnt = nullptr, *d_part_off = nullptr, *d_totals = nullptr;
  long long work_cap = 0;
  int grid = 1;
  // adjoint (allocated on first use)
  bool adj_ready = false;
  bool adj_warm = false;       // start each adjoint CG from the previous call's lambda
  bool adj_lam_valid = false;  // d_lam holds a solution of this mesh
  double4 *d_lam = nullptr, *d_r = nullptr, *d_z = nullptr, *d_pa = nullptr, *d_pb = nullptr, *d_q = nullptr,
          *d_zw = nullptr;
  double *d_adiag = nullptr, *d_agrad = nullptr, *d_E = nullptr;
  double *d_part_rz = nullptr, *d_part_pq = nullptr, *d_part_f = nullptr;
  double* d_aio = nullptr;         // [2][nV][3] + [nT] staging for host adjoint outputs
  CgScal* d_cgs = nullptr;
  int cgs_cap = 0;
  CgStatus* d_cgst = nullptr;
  CgStatus* h_cgst = nullptr;      // pinned
  bool E_uploaded = false;
  // optional per-launch timing (HIP events on the context stream)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;  // (kind, index of the start event)
  int ev_used = 0;
  double prof_us[PNCG_PROF_KINDS] = {0};
  long long prof_n[PNCG_PROF_KINDS] = {0};
};

namespace {

constexpr long long kTileScan = 4096;   // scan tile of the broad phase (kBlock * 16)

int fail(pncg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, PNCG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

template <typename T>
int dmalloc(pncg_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(c, PNCG_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return PNCG_OK;
}

void dfree(pncg_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

void drop_graphs(pncg_ctx* c) {
  for (auto& g : c->rgraph) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
}

void free_all(pncg_ctx* c) {
  drop_graphs(c);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_n) (void)hipHostFree(c->h_n);
  if (c->h_cgst) (void)hipHostFree(c->h_cgst);
  c->h_status = nullptr;
  c->h_n = nullptr;
  c->h_cgst = nullptr;
}

int ensure_device(pncg_ctx* c) {
  if (c->dev_ready) return PNCG_OK;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(c, PNCG_E_HIP, "no HIP device available");
  if (c->device < 0 || c->device >= n) return fail(c, PNCG_E_INVAL, "device ordinal out of range");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, scratch_address(c->device, &c->d_static));
  if (!c->stream) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  HIPCHK(c, hipHostMalloc((void**)&c->h_status, 2 * sizeof(StepStatus), hipHostMallocDefault));
  for (int i = 0; i < 2; ++i) HIPCHK(c, hipEventCreateWithFlags(&c->st_ev[i], hipEventDisableTiming));
  HIPCHK(c, hipHostMalloc((void**)&c->h_n, 4 * sizeof(long long), hipHostMallocDefault));
  c->dev_ready = true;
  return PNCG_OK;
}

int sync(pncg_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PNCG_OK;
}

template <typename R>
Args<R> make_args(pncg_ctx* c, double h) {
  Args<R> A{};
  A.nV = c->nV;
  A.nT = c->nT;
  A.elem = reinterpret_cast<const ElemRec<R>*>(c->d_elem);
  A.inc = c->d_inc;
  A.inc_vert = c->d_inc_vert;
  A.nWaves = c->nWaves;
  A.mass = c->d_mass;
  A.vflag = c->d_vflag;
  A.target = c->d_target;
  A.xbuild = c->d_xbuild;
  A.x0 = c->d_x0;
  A.x1 = c->d_x1;
  A.xt = c->d_xt;
  A.xstart = c->d_xstart;
  A.g = reinterpret_cast<R4<R>*>(c->d_g);
  A.pg = reinterpret_cast<R4<R>*>(c->d_pg);
  A.p0 = reinterpret_cast<R4<R>*>(c->d_p0);
  A.p1 = reinterpret_cast<R4<R>*>(c->d_p1);
  A.acc = c->d_acc;
  A.seg = c->scatter == PNCG_SCATTER_SEGMENTED ? 1 : 0;
  A.coff = c->d_coff;
  A.cent = c->d_cent;
  A.wrange = c->d_wrange;
  A.rp = c->d_rp;
  A.pv = A.seg ? c->d_pv : nullptr;
  A.self = (c->cflags & PNCG_CONTACT_SELF) && c->nF + c->nE > 0 ? 1 : 0;
  A.cand = c->d_cand;
  A.ncand = c->d_ncand;
  A.cand_cap = c->cand_cap;
  A.tris = c->d_tris;
  A.edges = c->d_edges;
  A.planes = c->planes;
  A.dhat = c->dhat;
  A.kappa = c->kappa;
  A.h = h;
  A.h2 = h * h;
  A.skin = c->skin;
  A.has_prims = (c->planes.n > 0 || A.self) ? 1 : 0;
  A.iter_max = c->iter_max;
  A.term = c->term;
  A.eps = c->eps;
  A.flags = c->sflags;
  A.scal = c->d_scal;
  A.status = c->d_status;
  A.part_grad = c->d_part_grad;
  A.part_dir = c->d_part_dir;
  A.part_narrow = c->d_part_narrow;
  A.grid = c->grid;
  A.split = (c->sflags & PNCG_SPLIT_OBJECTS) ? 1 : 0;
  A.nObj = c->nObj;
  A.model = kernel_model(c->model);
  A.vobj = c->d_vobj;
  A.voff = c->d_voff;
  A.toff = c->d_toff;
  A.oscal = c->d_oscal;
  A.vdots = c->d_vdots;
  A.tphp = c->d_tphp;
  A.vphp = c->d_vphp;
  A.opair = c->d_opair;
  return A;
}

// Point the list-dependent arguments at the current candidate list and its
// segmented-scatter arrays (a list build may reallocate them); E_STATE if
// the segmented arrays are missing where a kernel would use them.
template <typename R>
int list_args(pncg_ctx* c, Args<R>& A) {
  A.cand = c->d_cand;
  A.cand_cap = c->cand_cap;
  A.coff = c->d_coff;
  A.cent = c->d_cent;
  A.wrange = c->d_wrange;
  A.rp = c->d_rp;
  A.pv = A.seg ? c->d_pv : nullptr;
  if (A.self && A.seg && (!A.cand || !A.coff || !A.cent || !A.rp || !A.wrange || !A.pv))
    return fail(c, PNCG_E_STATE, "internal: the candidate list or its pair index is not allocated");
  return PNCG_OK;
}

Broad make_broad(pncg_ctx* c) {
  Broad B{};
  B.nV = c->nV;
  B.nSV = c->nSV;
  B.nF = c->nF;
  B.nE = c->nE;
  B.surf = c->d_surf;
  B.tris = c->d_tris;
  B.edges = c->d_edges;
  B.oid = c->d_oid;
  B.excl_pt = c->d_excl_pt;
  B.n_excl_pt = c->n_excl_pt;
  B.excl_ee = c->d_excl_ee;
  B.n_excl_ee = c->n_excl_ee;
  B.item_lo = c->d_item_lo;
  B.item_hi = c->d_item_hi;
  B.item_cnt = c->d_item_cnt;
  B.item_off = c->d_item_off;
  B.ent_cap = c->ent_cap;
  B.ent_key = c->d_ent_key;
  B.ent_item = c->d_ent_item;
  B.ent_rank = c->d_ent_rank;
  B.bkt_key = c->d_bkt_key;
  B.bkt_item = c->d_bkt_item;
  B.bkt_lo = c->d_bkt_lo;
  B.bkt_hi = c->d_bkt_hi;
  B.bkt_ids = c->d_bkt_ids;
  B.tsize = c->tsize;
  B.count = c->d_count;
  B.start = c->d_start;
  B.work_cap = c->work_cap;
  B.part_cnt = c->d_part_cnt;
  B.part_off = c->d_part_off;
  B.totals = c->d_totals;
  B.grid = c->grid;
  return B;
}

PairIndex make_pairindex(pncg_ctx* c) {
  PairIndex P{};
  P.nV = c->nV;
  P.tris = c->d_tris;
  P.edges = c->d_edges;
  P.vcnt = c->d_vcnt;
  P.coff = c->d_coff;
  P.cent = c->d_cent;
  P.cent_tmp = c->d_cent_tmp;
  P.ckey_tmp = c->d_ckey_tmp;
  P.pv = c->d_pv;
  P.big = c->d_big;
  P.scan_tmp = c->d_pl_tmp;
  P.wvert = c->d_wvert;
  P.wrange = c->d_wrange;
  P.nWaves = c->nWaves;
  P.grid = c->grid;
  return P;
}

// Capacity of the candidate list and of the arrays sized by it (the sort
// buffer, corner entries, activity flags and slots of the segmented
// scatter); contents are not kept.
int ensure_cand_cap(pncg_ctx* c, long long cap) {
  if (cap <= c->cand_cap) return PNCG_OK;
  if (c->noalloc)
    return fail(c, PNCG_E_CAPACITY, "the candidate list needs larger buffers (a pncg_step_dev call grows them)");
  drop_graphs(c);
  c->list_valid = false;
  for (void* p : {(void*)c->d_cand, (void*)c->d_cent, (void*)c->d_cent_tmp, (void*)c->d_ckey_tmp, (void*)c->d_rp,
                  (void*)c->d_pv})
    dfree(c, p);
  c->d_cand = nullptr;
  c->d_pv = nullptr;
  c->d_ckey_tmp = nullptr;
  c->d_cent = c->d_cent_tmp = nullptr;
  c->d_rp = nullptr;
  c->cand_cap = 0;
  int rc;
  if ((rc = dmalloc(c, &c->d_cand, (size_t)cap))) return rc;
  if (c->scatter == PNCG_SCATTER_SEGMENTED &&
      ((rc = dmalloc(c, &c->d_cent, 4 * (size_t)cap)) || (rc = dmalloc(c, &c->d_cent_tmp, 4 * (size_t)cap)) ||
       (rc = dmalloc(c, &c->d_ckey_tmp, 4 * (size_t)cap)) ||
       (rc = dmalloc(c, &c->d_rp, 24 * (size_t)cap)) || (rc = dmalloc(c, &c->d_pv, (size_t)cap))))
    return rc;
  c->cand_cap = cap;
  return PNCG_OK;
}

bool self_contact(const pncg_ctx* c) { return (c->cflags & PNCG_CONTACT_SELF) && c->nF + c->nE > 0; }

// The override lists (pncg_set_candidates_override) as one device list.
int upload_override(pncg_ctx* c) {
  if (c->ovr_uploaded) return PNCG_OK;
  if (c->noalloc) return fail(c, PNCG_E_STATE, "internal: the candidate override was not uploaded");
  std::vector<int2> all(c->ovr[0]);
  for (const int2& e : c->ovr[1]) all.push_back(make_int2(e.x, ~e.y));
  dfree(c, c->d_ovr);
  c->d_ovr = nullptr;
  int rc;
  if ((rc = dmalloc(c, &c->d_ovr, all.size()))) return rc;
  if (!all.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_ovr, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, c->stream));
  c->n_ovr = (long long)all.size();
  c->ovr_uploaded = true;
  return PNCG_OK;
}

// With the segmented scatter, index the corner entries of the list in d_cand.
void finish_list(pncg_ctx* c) {
  if (c->scatter != PNCG_SCATTER_SEGMENTED) return;
  pairs_index(make_pairindex(c), c->d_cand, c->d_ncand, c->cand_cap, c->stream);
}

// The override as the current candidate list (kind in the pair).
int install_override(pncg_ctx* c) {
  int rc;
  c->list_valid = false;
  if ((rc = upload_override(c))) return rc;
  if ((rc = ensure_cand_cap(c, std::max<long long>(c->n_ovr, 1024)))) return rc;
  pairs_install(c->d_ovr, c->n_ovr, c->d_cand, c->d_ncand, &c->d_status->n_cand, c->stream);
  finish_list(c);
  return PNCG_OK;
}

// (Re)allocate the cell-entry arrays for `ent` entries and the hash table and
// work arrays that depend on it.
int alloc_grid(pncg_ctx* c, long long ent) {
  int rc;
  drop_graphs(c);
  for (void* p : {(void*)c->d_ent_key, (void*)c->d_ent_item, (void*)c->d_ent_rank, (void*)c->d_bkt_key,
                  (void*)c->d_bkt_item,
                  (void*)c->d_bkt_lo, (void*)c->d_bkt_hi, (void*)c->d_bkt_ids, (void*)c->d_count,
                  (void*)c->d_start, (void*)c->d_part_cnt, (void*)c->d_part_off})
    dfree(c, p);
  c->ent_cap = std::max<long long>(ent, 4096);
  int ts = 1024;
  while (ts < c->ent_cap / 4 && ts < (1 << 24)) ts <<= 1;
  c->tsize = ts;
  c->work_cap = (long long)c->nSV + c->ent_cap;
  if ((rc = dmalloc(c, &c->d_ent_key, c->ent_cap)) || (rc = dmalloc(c, &c->d_ent_item, c->ent_cap)) ||
      (rc = dmalloc(c, &c->d_ent_rank, c->ent_cap)) ||
      (rc = dmalloc(c, &c->d_bkt_key, c->ent_cap)) || (rc = dmalloc(c, &c->d_bkt_item, c->ent_cap)) ||
      (rc = dmalloc(c, &c->d_bkt_lo, c->ent_cap)) || (rc = dmalloc(c, &c->d_bkt_hi, c->ent_cap)) ||
      (rc = dmalloc(c, &c->d_bkt_ids, c->ent_cap)) ||
      (rc = dmalloc(c, &c->d_count, ts)) || (rc = dmalloc(c, &c->d_start, ts + 1)) ||
      (rc = dmalloc(c, &c->d_part_cnt, c->work_cap)) || (rc = dmalloc(c, &c->d_part_off, c->work_cap + 4096)))
    return rc;
  return PNCG_OK;
}

__global__ void k_copy_counts(const long long* totals, long long* ncand) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ncand[0] = totals[1];
    ncand[1] = totals[2];
  }
}

// Candidate pairs (PT then EE) at device positions x with inflation r into
// c->d_cand; counts in c->d_ncand.  filter_d >= 0: same-object pairs closer
// than filter_d only (rest-pose exclusion set).  One host synchronisation
// (to size the pair list); the grid is rebuilt larger if its entry capacity
// was too small.
int build_candidates(pncg_ctx* c, const double4* x, double r, double filter_d, int filter_obj, long long* n_total,
                     long long* n_pt, bool indexed = false) {
  int rc;
  c->list_valid = false;   // the candidate buffer no longer holds the solver's list
  long long n = 0;
  for (int attempt = 0; attempt < 3; ++attempt) {
    Broad B = make_broad(c);
    broad_build_count(B, x, c->cell, r, filter_d, filter_obj, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->h_n, c->d_totals, 3 * sizeof(long long), hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync(c))) return rc;
    if (c->h_n[0] <= c->ent_cap) break;
    if ((rc = alloc_grid(c, c->h_n[0] + c->h_n[0] / 4))) return rc;
  }
  if (c->h_n[0] > c->ent_cap) return fail(c, PNCG_E_NOMEM, "spatial grid did not fit");
  n = c->h_n[1];
  const long long npt = c->h_n[2];
  hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, c->stream, (const long long*)c->d_totals, c->d_ncand);
  if ((n > c->cand_cap || c->cand_cap == 0) && (rc = ensure_cand_cap(c, std::max<long long>(n + n / 2, 1024))))
    return rc;
  broad_fill(make_broad(c), x, c->cell, r, filter_d, filter_obj, c->d_cand, c->cand_cap, c->stream);
  if (indexed) finish_list(c);
  if (n_total) *n_total = n;
  if (n_pt) *n_pt = npt;
  return PNCG_OK;
}

constexpr int kRestart = 1000;   // internal: a capacity was exceeded, run the step again

// The solver's candidate list at device positions x (pairs within
// dhat + skin, unordered, kind in the pair), built without host
// synchronisation; a grid or list that did not fit raises kErrCapacity in
// the step status, which the step loop turns into a rerun with larger
// buffers.  Also records the build positions.
int build_solver_list(pncg_ctx* c, const double4* x) {
  int rc;
  if (c->ovr_set[0] || c->ovr_set[1]) {
    if ((rc = install_override(c))) return rc;
    copy_positions(c->d_xbuild, x, c->nV, c->stream);
    return PNCG_OK;
  }
  if ((rc = ensure_cand_cap(c, std::max<long long>(4096, 2LL * c->nSV)))) return rc;
  const Broad B = make_broad(c);
  const PairIndex P = make_pairindex(c);
  const double r = c->dhat + c->skin;
  const bool seg = c->scatter == PNCG_SCATTER_SEGMENTED;
  auto enqueue = [&]() {
    broad_solver_list(B, x, c->cell, r, c->d_cand, c->cand_cap, c->d_ncand, &c->d_status->err,
                      &c->d_status->n_cand, c->stream, seg ? &P : nullptr, c->d_xbuild);
    if (seg) pairs_index(P, c->d_cand, c->d_ncand, c->cand_cap, c->stream, true);
  };
  if (!c->graphs || c->noalloc) {
    enqueue();
    return PNCG_OK;
  }
  // Everything the launches take by value or by address, as one byte image:
  // a graph is replayed only while all of it is unchanged.
  auto& g = c->rgraph[x == c->d_x1 ? 1 : 0];
  unsigned char key[sizeof g.key] = {};
  const void* ptrs[8] = {x, c->d_cand, c->d_ncand, c->d_status, c->d_xbuild, c->stream, nullptr, nullptr};
  const double vals[4] = {c->cell, r, (double)c->cand_cap, (double)c->scatter};
  std::memcpy(key, &B, sizeof B);
  std::memcpy(key + sizeof B, &P, sizeof P);
  std::memcpy(key + sizeof B + sizeof P, ptrs, sizeof ptrs);
  std::memcpy(key + sizeof B + sizeof P + sizeof ptrs, vals, sizeof vals);
  if (!g.exec || std::memcmp(key, g.key, sizeof key) != 0) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    enqueue();
    hipGraph_t graph = nullptr;
    HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return fail(c, PNCG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    std::memcpy(g.key, key, sizeof key);
  }
  HIPCHK(c, hipGraphLaunch(g.exec, c->stream));
  return PNCG_OK;
}

// After a kRestart: size the grid and the list for what the last build found.
int grow_solver_buffers(pncg_ctx* c) {
  long long cnt[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(&cnt[0], c->d_totals, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&cnt[1], c->d_ncand, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
  int rc = sync(c);
  if (rc) return rc;
  if (cnt[0] > c->ent_cap && (rc = alloc_grid(c, cnt[0] + cnt[0] / 2))) return rc;
  if (cnt[1] > c->cand_cap && (rc = ensure_cand_cap(c, cnt[1] + cnt[1] / 2 + 1024))) return rc;
  return PNCG_OK;
}

int upload_rows(pncg_ctx* c, const double* host, double* dev, int n) {
  HIPCHK(c, hipMemcpyAsync(dev, host, sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, c->stream));
  return PNCG_OK;
}

__global__ void k_rows_to_x4(const double* a, double4* x, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = make_double4(a[3 * i], a[3 * i + 1], a[3 * i + 2], 0.0);
}

int check_status_err(pncg_ctx* c, const StepStatus& st) {
  if (st.err & kErrNonfinite) return fail(c, PNCG_E_NONFINITE, "non-finite value in positions or velocities");
  if (st.err & kErrInverted) return fail(c, PNCG_E_INVERTED, inverted_message(c->model));
  if (st.err & kErrPenetration) return fail(c, PNCG_E_PENETRATION, "a contact distance is <= 0");
  return PNCG_OK;
}

// ------------------------------------------------------------- profiling
int prof_begin(pncg_ctx* c, int kind) {
  if (!c->profiling) return -1;
  if (c->ev_used + 2 > (int)c->ev_pool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->ev_pool.push_back(e);
    }
  }
  const int i = c->ev_used;
  c->ev_used += 2;
  (void)hipEventRecord(c->ev_pool[i], c->stream);
  c->ev_pending.push_back({kind, i});
  return i;
}
void prof_end(pncg_ctx* c, int i) {
  if (i < 0) return;
  (void)hipEventRecord(c->ev_pool[i + 1], c->stream);
}
// after a stream synchronisation: fold the recorded pairs into the totals
void prof_collect(pncg_ctx* c) {
  for (auto& pe : c->ev_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev_pool[pe.second], c->ev_pool[pe.second + 1]) == hipSuccess) {
      c->prof_us[pe.first] += 1000.0 * ms;
      c->prof_n[pe.first] += 1;
    }
  }
  c->ev_pending.clear();
  c->ev_used = 0;
}

// Copy the step status into pinned slot `slot` behind the work enqueued so
// far, and mark it with that slot's event.
int enqueue_status(pncg_ctx* c, int slot) {
  HIPCHK(c, hipMemcpyAsync(c->h_status + slot, c->d_status, sizeof(StepStatus), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->st_ev[slot], c->stream));
  return PNCG_OK;
}
// Wait for slot's copy (and everything enqueued before it).
int wait_status(pncg_ctx* c, int slot) {
  HIPCHK(c, hipEventSynchronize(c->st_ev[slot]));
  if (c->profiling) prof_collect(c);
  return PNCG_OK;
}

int read_status(pncg_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, c->d_status, sizeof(StepStatus), hipMemcpyDeviceToHost, c->stream));
  int rc = sync(c);
  if (c->profiling) prof_collect(c);
  return rc;
}

// ------------------------------------------------------------------ step
// sync_end = false (the steps of pncg_run_dev but its last): the step ends as
// soon as a chunk's status shows the stop, with the output kernel queued and
// no further host wait, so that the next step's launches follow at once; its
// statistics are the stopping status.  A non-finite result, which only the
// output kernel would flag, is then found by the next step's predictor.
template <typename R>
int step_impl(pncg_ctx* c, const double* x_dev, const double* v_dev, double h, double* x_out, double* v_out,
              pncg_stats* st, bool sync_end = true) {
  Args<R> A = make_args<R>(c, h);
  const double3 grav = make_double3(c->grav[0], c->grav[1], c->grav[2]);
  // The solver's list: pairs within dhat + skin at the build positions (a
  // pair's distance changes by at most twice the per-vertex displacement,
  // which stays below skin / 2 until the next build).  A step may start on
  // the list the previous step of this context left, if that step ended
  // with at most a quarter of the skin used: the predictor then measures x_0
  // against the list's build positions and iteration 0 pauses for a rebuild
  // if the list no longer covers x_0 (the caller may pass any state).
  const bool carry = A.self && c->list_valid && !(c->ovr_set[0] || c->ovr_set[1]) &&
                     c->last_D_end <= 0.25 * c->skin;
  c->list_valid = false;
  A.carry = carry ? 1 : 0;
  int ev = prof_begin(c, PNCG_PROF_PREDICT);
  launch_predict<R>(A, x_dev, v_dev, grav, c->stream);
  prof_end(c, ev);
  int rebuilds = 0;
  int rc;
  if (A.self) {
    if (!carry) {
      ev = prof_begin(c, PNCG_PROF_REBUILD);
      if ((rc = build_solver_list(c, c->d_x0))) return rc;
      prof_end(c, ev);
      ++rebuilds;
    }
    if ((rc = list_args(c, A))) return rc;
  }
  // With self contact the chunk length is chosen so that the displacement
  // bound is expected to stay inside half the skin (observed growth per
  // iteration, starting from the worst case dhat / 2); the device pauses the
  // chunk if the prediction fails.
  double D = carry ? c->last_D_end : 0.0, rate = 0.5 * c->dhat;
  auto chunk_len = [&](double Dpred) {
    int m = c->chunk;
    if (A.self) {
      const double room = 0.5 * c->skin - Dpred;
      const double want = room / std::max(rate, 1e-300);
      m = (int)std::min<double>(std::max<double>(std::floor(want), 1.0), (double)c->chunk);
    }
    return m;
  };
  // Enqueue iterations [k0, k0 + m) (the last launch of the cap finishes the
  // step); returns the end of the chunk.
  // A chunk that reaches the cap ends the step whatever happens before it
  // (unless a pause comes first), so the output kernel goes right behind it;
  // it reads the final iteration from the device status and writes only if
  // the step has stopped without an error (so outputs that alias the inputs,
  // which a capacity rerun reads again, stay intact), and a later one
  // supersedes it if the step resumes.
  const bool early_final = true;
  bool last_is_final = false;
  auto launch_chunk = [&](int k0, int m, int mode0) {
    // fold the pair pass into the sweep while the last list had at most one
    // corner entry per vertex on average (sparse contact)
    A.fuse = 4 * c->last_ncand <= (long long)c->nV ? 1 : 0;
    const bool fused = fused_pairs(A);
    const int kind_first = (A.self && !fused) ? PNCG_PROF_NARROW : PNCG_PROF_GRAD;
    const int kend = std::min(k0 + m, c->iter_max + 1);
    last_is_final = false;
    for (int j = k0; j < kend; ++j) {
      int e = prof_begin(c, kind_first);
      if (j == c->iter_max) {
        launch_iteration_first<R>(A, j, 1 /*finish*/, c->stream);
        prof_end(c, e);
        break;
      }
      launch_iteration_first<R>(A, j, (j == k0) ? mode0 : 0, c->stream);
      prof_end(c, e);
      if (A.self && !fused) {
        e = prof_begin(c, PNCG_PROF_GRAD);
        launch_iteration_grad<R>(A, j, c->stream);
        prof_end(c, e);
      }
      e = prof_begin(c, PNCG_PROF_DIR);
      launch_iteration_dir<R>(A, j, c->stream);
      prof_end(c, e);
    }
    if (early_final && kend == c->iter_max + 1) {
      const int e = prof_begin(c, PNCG_PROF_PREDICT);
      launch_finalize<R>(A, x_out, v_out, c->stream);
      prof_end(c, e);
      last_is_final = true;
    }
    return kend;
  };
  // One chunk stays in flight while the status of the one before it is read,
  // so the device does not idle across the host's round trip.  Launches after
  // a stop or a pause do nothing (each iteration's first kernel sees its
  // predecessor's flag), and a resume rewrites the paused iteration's
  // scalars, so a chunk sent ahead is harmless.  With profiling on, chunks go
  // one at a time so that every recorded event pair has completed when the
  // totals are collected.
  const bool ahead = !c->profiling;
  auto bail = [&](int code) {
    (void)hipStreamSynchronize(c->stream);
    return code;
  };
  int k = 0, cur = 0;
  StepStatus last_s{};
  int kend = launch_chunk(0, chunk_len(D), 0 /*kModeNormal*/);
  if ((rc = enqueue_status(c, cur))) return rc;
  while (true) {
    int kn = -1;
    if (ahead && kend <= c->iter_max) {
      kn = launch_chunk(kend, chunk_len(D + rate * (kend - k)), 0);
      if ((rc = enqueue_status(c, cur ^ 1))) return bail(rc);
    }
    if ((rc = wait_status(c, cur))) return bail(rc);
    const StepStatus s = c->h_status[cur];
    last_s = s;
    if (A.self) c->last_ncand = s.n_cand;
    if (s.err & kErrCapacity) return bail(kRestart);
    if ((rc = check_status_err(c, s))) return bail(rc);
    if (s.stopped) break;
    if (s.paused_at >= 0) {
      const int p = s.paused_at;
      int e = prof_begin(c, PNCG_PROF_REBUILD);
      last_is_final = false;
      if ((rc = build_solver_list(c, (p & 1) ? c->d_x1 : c->d_x0))) return bail(rc);
      prof_end(c, e);
      ++rebuilds;
      if ((rc = list_args(c, A))) return bail(rc);
      if (p > k) rate = std::max(rate, (s.D - D) / (p - k + 1));
      D = 0.0;
      k = p;
      kend = launch_chunk(k, chunk_len(D), 2 /*kModeResume*/);
      if ((rc = enqueue_status(c, cur))) return bail(rc);
      continue;
    }
    if (kend > k) rate = std::max(0.0, (s.D - D) / (kend - k));
    D = s.D;
    k = kend;
    if (kn >= 0) {
      kend = kn;
      cur ^= 1;
    } else {
      kend = launch_chunk(k, chunk_len(D), 0);
      if ((rc = enqueue_status(c, cur))) return bail(rc);
    }
  }
  if (!last_is_final) {
    ev = prof_begin(c, PNCG_PROF_PREDICT);
    launch_finalize<R>(A, x_out, v_out, c->stream);
    prof_end(c, ev);
  }
  StepStatus s = last_s;
  if (sync_end) {
    if ((rc = read_status(c))) return rc;
    s = *c->h_status;
    if ((rc = check_status_err(c, s))) return rc;
  }
  if (A.self) {
    // the list and its build positions stay for the next step
    c->list_valid = true;
    c->last_D_end = s.D;
  }
  if (st) {
    st->iters = s.iters;
    st->reason = s.reason;
    st->dE0 = s.dE0;
    st->last_dE = s.last_dE;
    st->g0_norm = s.g0;
    st->g_norm = s.gk;
    st->alpha_upper_hits = s.a_up_hits;
    st->rebuilds = rebuilds;
    st->n_candidates = A.self ? s.n_cand : 0;
    st->n_active = (long long)s.n_active;
  }
  return s.reason == 2 ? PNCG_W_MAXITER : PNCG_OK;
}

int ready(pncg_ctx* c) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 2) return fail(c, PNCG_E_STATE, "set_mesh and set_material must come first");
  return PNCG_OK;
}

// Ensure the candidate buffer reflects r at device positions in d_x0.
int query_candidates(pncg_ctx* c, double r) {
  if (!self_contact(c)) return PNCG_OK;
  if (c->ovr_set[0] || c->ovr_set[1]) return install_override(c);
  return build_candidates(c, c->d_x0, r, r, 0, nullptr, nullptr, true);
}

int stage_positions(pncg_ctx* c, const double* x) {
  if (!finite_all(x, 3 * (size_t)c->nV)) return fail(c, PNCG_E_NONFINITE, "non-finite position");
  int rc = upload_rows(c, x, c->d_io, c->nV);
  if (rc) return rc;
  hipLaunchKernelGGL(k_rows_to_x4, dim3(c->grid), dim3(kBlock), 0, c->stream, (const double*)c->d_io, c->d_x0, c->nV);
  return PNCG_OK;
}

template <typename R>
int load_query(pncg_ctx* c, const double* x, const double* xt, const double* p) {
  const size_t n3 = 3 * (size_t)c->nV;
  if (!finite_all(x, n3) || (xt && !finite_all(xt, n3)) || (p && !finite_all(p, n3)))
    return fail(c, PNCG_E_NONFINITE, "non-finite input");
  int rc;
  if ((rc = upload_rows(c, x, c->d_io, c->nV))) return rc;
  if (xt && (rc = upload_rows(c, xt, c->d_io + n3, c->nV))) return rc;
  if (p && (rc = upload_rows(c, p, c->d_io + 2 * n3, c->nV))) return rc;
  Args<R> A = make_args<R>(c, 1.0);
  launch_load_query<R>(A, c->d_io, xt ? c->d_io + n3 : nullptr, p ? c->d_io + 2 * n3 : nullptr, c->stream);
  return query_candidates(c, c->dhat);
}

int finish_query(pncg_ctx* c) {
  int rc = read_status(c);
  if (rc) return rc;
  return check_status_err(c, *c->h_status);
}

template <typename R>
int energy_impl(pncg_ctx* c, const double* x, const double* xt, double h, double* out) {
  int rc = load_query<R>(c, x, xt, nullptr);
  if (rc) return rc;
  Args<R> A = make_args<R>(c, h);
  if ((rc = list_args(c, A))) return rc;
  launch_query_energy<R>(A, c->d_scalar, c->stream);
  HIPCHK(c, hipMemcpyAsync(out, c->d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return finish_query(c);
}

template <typename R>
int gradient_impl(pncg_ctx* c, const double* x, const double* xt, double h, double* g, double* d) {
  int rc = load_query<R>(c, x, xt, nullptr);
  if (rc) return rc;
  Args<R> A = make_args<R>(c, h);
  if ((rc = list_args(c, A))) return rc;
  const size_t n3 = 3 * (size_t)c->nV;
  double* dg = c->d_io;          // x staging is no longer needed
  double* dd = c->d_io + 2 * n3;
  launch_query_gradient<R>(A, dg, d ? dd : nullptr, c->stream);
  HIPCHK(c, hipMemcpyAsync(g, dg, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  if (d) HIPCHK(c, hipMemcpyAsync(d, dd, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  return finish_query(c);
}

template <typename R>
int hvp_impl(pncg_ctx* c, const double* x, const double* p, double h, double* hp, double* php) {
  int rc = load_query<R>(c, x, nullptr, p);
  if (rc) return rc;
  Args<R> A = make_args<R>(c, h);
  if ((rc = list_args(c, A))) return rc;
  const size_t n3 = 3 * (size_t)c->nV;
  double* dh = c->d_io + n3;
  launch_query_hvp<R>(A, hp ? dh : nullptr, c->d_scalar, c->stream);
  if (hp) HIPCHK(c, hipMemcpyAsync(hp, dh, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(php, c->d_scalar, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return finish_query(c);
}

template <typename R>
int upload_elements(pncg_ctx* c) {
  std::vector<ElemRec<R>> rec(c->nT);
  for (int e = 0; e < c->nT; ++e) {
    ElemRec<R>& r = rec[e];
    for (int a = 0; a < 4; ++a) r.v[a] = c->tets[4 * e + a];
    for (int j = 0; j < 9; ++j) r.B[j] = R(c->Bm[9 * e + j]);
    const double mu = c->E[e] / (2.0 * (1.0 + c->nu[e]));
    const double lam = c->E[e] * c->nu[e] / ((1.0 + c->nu[e]) * (1.0 - 2.0 * c->nu[e]));
    r.vmu = R(c->vol[e] * mu);
    r.vlam = R(c->vol[e] * record_lam(c->model, mu, lam));
  }
  if (!c->d_elem) {
    int rc = dmalloc(c, reinterpret_cast<ElemRec<R>**>(&c->d_elem), (size_t)c->nT);
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpyAsync(c->d_elem, rec.data(), sizeof(ElemRec<R>) * (size_t)c->nT, hipMemcpyHostToDevice, c->stream));
  return sync(c);
}

int upload_flags_targets(pncg_ctx* c) {
  std::vector<uint8_t> fl(c->vflag);
  std::vector<double4> tg(c->nV, make_double4(0, 0, 0, 0));
  for (size_t i = 0; i < c->fixed.size(); ++i) {
    const int v = c->fixed[i];
    fl[v] |= kFixed;
    tg[v] = make_double4(c->fixed_target[3 * i], c->fixed_target[3 * i + 1], c->fixed_target[3 * i + 2], 0.0);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_vflag, fl.data(), c->nV, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_target, tg.data(), sizeof(double4) * c->nV, hipMemcpyHostToDevice, c->stream));
  return sync(c);
}

// ---------------------------------------------------------------- adjoint
int ensure_adjoint(pncg_ctx* c, int cg_max) {
  int rc;
  if (!c->adj_ready) {
    const size_t nV = c->nV, nT = c->nT;
    if ((rc = dmalloc(c, &c->d_lam, nV)) || (rc = dmalloc(c, &c->d_r, nV)) || (rc = dmalloc(c, &c->d_z, nV)) ||
        (rc = dmalloc(c, &c->d_pa, nV)) || (rc = dmalloc(c, &c->d_pb, nV)) || (rc = dmalloc(c, &c->d_q, nV)) ||
        (rc = dmalloc(c, &c->d_adiag, 3 * nV)) || (rc = dmalloc(c, &c->d_agrad, 3 * nV)) ||
        (rc = dmalloc(c, &c->d_E, nT)) || (rc = dmalloc(c, &c->d_part_rz, 2 * (size_t)kMaxGrid)) ||
        (rc = dmalloc(c, &c->d_part_pq, (size_t)kMaxGrid)) || (rc = dmalloc(c, &c->d_aio, 6 * nV + nT)) ||
        (rc = dmalloc(c, &c->d_cgst, 1)) || (rc = dmalloc(c, &c->d_zw, 4 * nV)) ||
        (rc = dmalloc(c, &c->d_part_f, 8 * (size_t)kMaxGrid)))
      return rc;
    if (!c->h_cgst) HIPCHK(c, hipHostMalloc((void**)&c->h_cgst, sizeof(CgStatus), hipHostMallocDefault));
    c->adj_ready = true;
  }
  if (c->cgs_cap < cg_max + 1) {
    if (c->d_cgs) dfree(c, c->d_cgs);
    c->d_cgs = nullptr;
    if ((rc = dmalloc(c, &c->d_cgs, (size_t)cg_max + 1))) return rc;
    c->cgs_cap = cg_max + 1;
  }
  if (!c->E_uploaded) {
    HIPCHK(c, hipMemcpyAsync(c->d_E, c->E.data(), sizeof(double) * c->nT, hipMemcpyHostToDevice, c->stream));
    c->E_uploaded = true;
  }
  return PNCG_OK;
}

// All pointers are device pointers.  Ebar is accumulated.
int adjoint_impl(pncg_ctx* c, const double* x1, double h, const double* xbar, const double* vbar, double cg_tol,
                 int cg_max, double* xbar_t, double* vbar_t, double* Ebar, pncg_adjoint_stats* st) {
  int rc;
  if ((rc = ensure_adjoint(c, cg_max))) return rc;
  Args<double> A = make_args<double>(c, h);
  launch_load_query<double>(A, x1, nullptr, nullptr, c->stream);
  if ((rc = query_candidates(c, c->dhat))) return rc;
  if ((rc = list_args(c, A))) return rc;
  // Jacobi diagonal of H at x^{t+1} (the gradient written alongside is
  // unused; the predictor is taken as x^{t+1} so that it stays finite)
  A.xt = c->d_x0;
  launch_query_gradient<double>(A, c->d_agrad, c->d_adiag, c->stream);
  A.xt = c->d_xt;
  AdjArgs C{};
  C.lam = c->d_lam;
  C.r = c->d_r;
  C.z = c->d_z;
  C.pbuf[0] = c->d_pa;
  C.pbuf[1] = c->d_pb;
  C.q = c->d_q;
  C.zw[0] = c->d_zw;
  C.zw[1] = c->d_zw + 2 * (size_t)c->nV;
  C.part_f = c->d_part_f;
  C.diag = c->d_adiag;
  C.part_rz = c->d_part_rz;
  C.part_pq = c->d_part_pq;
  C.scal = c->d_cgs;
  C.status = c->d_cgst;
  C.tol2 = cg_tol * cg_tol;
  C.max_iter = cg_max;
  const bool fused = !A.self;
  const bool warm = fused && c->adj_warm && c->adj_lam_valid;
  if (warm) HIPCHK(c, hipMemsetAsync(&c->d_cgst->stopped, 0, sizeof(int), c->stream));
  launch_adj_init(A, C, xbar, vbar, warm, c->stream);
  const int last = fused ? cg_max + 1 : cg_max;   // the launch that reports the end at the latest
  int k = 0, chunk = 16;
  while (true) {
    const int kend = std::min(k + chunk, last + 1);
    for (int j = k; j < kend; ++j) launch_cg_iteration(A, C, j, fused, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->h_cgst, c->d_cgst, sizeof(CgStatus), hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync(c))) return rc;
    if (c->h_cgst->stopped) break;
    if (kend > last) return fail(c, PNCG_E_HIP, "adjoint CG did not report its end");
    k = kend;
    chunk = std::min(chunk * 2, 256);
  }
  const CgStatus cs = *c->h_cgst;
  if (st) {
    st->cg_iters = cs.iters;
    st->reason = cs.reason;
    st->rel_residual = cs.bb > 0.0 ? std::sqrt(cs.rr / cs.bb) : 0.0;
  }
  if (cs.reason == 2) {
    c->adj_lam_valid = false;
    return fail(c, PNCG_E_INDEFINITE, "p^T H p <= 0 or not finite in the adjoint CG");
  }
  c->adj_lam_valid = true;
  launch_adj_out(A, C, vbar, c->d_E, xbar_t, vbar_t, Ebar, c->stream);
  if ((rc = read_status(c))) return rc;
  if ((rc = check_status_err(c, *c->h_status))) return rc;
  return cs.reason == 1 ? PNCG_W_MAXITER : PNCG_OK;
}

int adjoint_checks(pncg_ctx* c, const void* x1, double h, const void* xbar, const void* vbar, double cg_tol,
                   int cg_max, const void* xbar_t, const void* vbar_t, const void* Ebar) {
  int rc = ready(c);
  if (rc) return rc;
  if (c->precision != PNCG_FP64) return fail(c, PNCG_E_STATE, "the adjoint needs a PNCG_FP64 context");
  if (!x1 || !xbar || !vbar || !xbar_t || !vbar_t || !Ebar) return fail(c, PNCG_E_INVAL, "NULL argument");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  if (!(cg_tol >= 0.0) || !std::isfinite(cg_tol) || cg_max < 1) return fail(c, PNCG_E_INVAL, "need cg_tol >= 0, cg_max >= 1");
  return PNCG_OK;
}

// Verlet skin of the solver's candidate list: large enough that the list
// lasts many iterations, small against the mesh spacing so that neighbouring
// primitives of one surface (never active, a fraction of an edge apart) stay
// out of it: 0.4 of the mean surface edge less dhat, within [2, 8] dhat.
double default_skin(double dhat, double lmean) {
  if (!(lmean > 0.0)) return 4.0 * dhat;
  return std::min(8.0 * dhat, std::max(2.0 * dhat, 0.4 * lmean - dhat));
}

int grid_for(const pncg_ctx* c) {
  long long work = std::max<long long>({(long long)c->nWaves * kWave, (long long)c->nT, (long long)c->nV, 1LL});
  long long g = (work + kSBlock - 1) / kSBlock;
  g = std::min<long long>(std::max<long long>(g, 1), kMaxGrid);
  return (int)(((g + kXcds - 1) / kXcds) * kXcds);   // whole rounds over the XCDs
}

}  // namespace

// =================================================================== C ABI
// Objects of the split step must be contiguous vertex ranges (non-decreasing
// ids) whose tets are contiguous too; the reason if not, else NULL.
static const char* split_layout_error(const pncg_ctx* c) {
  for (int v = 1; v < c->nV; ++v)
    if (c->oid[v] < c->oid[v - 1]) return "splitting needs object ids non-decreasing over the vertices";
  int prev = INT_MIN;
  for (int e = 0; e < c->nT; ++e) {
    const int o = c->oid[c->tets[4 * e]];
    for (int a = 1; a < 4; ++a)
      if (c->oid[c->tets[4 * e + a]] != o) return "splitting: a tet spans two objects";
    if (o < prev) return "splitting needs the tets grouped by object in object order";
    prev = o;
  }
  return nullptr;
}

extern "C" {

int pncg_create(pncg_ctx** out, const pncg_opts* o) {
  if (!out) {
    g_create_error = "out is NULL";
    return PNCG_E_INVAL;
  }
  *out = nullptr;
  pncg_ctx* c = new (std::nothrow) pncg_ctx();
  if (!c) {
    g_create_error = "out of host memory";
    return PNCG_E_NOMEM;
  }
  if (o) {
    if (o->precision != PNCG_FP64 && o->precision != PNCG_MIXED) {
      delete c;
      g_create_error = "precision must be PNCG_FP64 or PNCG_MIXED";
      return PNCG_E_INVAL;
    }
    if (o->device < 0 || o->chunk < 0) {
      delete c;
      g_create_error = "negative device or chunk";
      return PNCG_E_INVAL;
    }
    if (o->scatter < PNCG_SCATTER_AUTO || o->scatter > PNCG_SCATTER_SEGMENTED) {
      delete c;
      g_create_error = "scatter must be PNCG_SCATTER_AUTO, _ATOMIC or _SEGMENTED";
      return PNCG_E_INVAL;
    }
    if (o->graphs != 0 && o->graphs != 1) {
      delete c;
      g_create_error = "graphs must be 0 or 1";
      return PNCG_E_INVAL;
    }
    c->graphs = o->graphs == 0;
    c->scatter = o->scatter == PNCG_SCATTER_ATOMIC ? PNCG_SCATTER_ATOMIC : PNCG_SCATTER_SEGMENTED;
    c->device = o->device;
    c->precision = o->precision;
    c->stream = reinterpret_cast<hipStream_t>(o->stream);
    if (o->chunk > 0) c->chunk = o->chunk;
  }
  *out = c;
  return PNCG_OK;
}

void pncg_destroy(pncg_ctx* c) {
  if (!c) return;
  if (c->dev_ready) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->st_ev)
      if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* pncg_last_error(const pncg_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

int pncg_set_mesh(pncg_ctx* c, int32_t nV, const double* X, int32_t nT, const int32_t* tets, int32_t nF,
                  const int32_t* tris, int32_t nE, const int32_t* edges, const int32_t* object_id) {
  if (!c) return PNCG_E_INVAL;
  if (nV <= 0 || nT <= 0 || nF < 0 || nE < 0 || !X || !tets || (nF > 0 && !tris) || (nE > 0 && !edges))
    return fail(c, PNCG_E_INVAL, "bad mesh sizes or NULL arrays");
  if (!finite_all(X, 3 * (size_t)nV)) return fail(c, PNCG_E_NONFINITE, "non-finite rest position");
  for (long long i = 0; i < 4LL * nT; ++i)
    if (tets[i] < 0 || tets[i] >= nV) return fail(c, PNCG_E_INVAL, "tet index out of range");
  for (long long i = 0; i < 3LL * nF; ++i)
    if (tris[i] < 0 || tris[i] >= nV) return fail(c, PNCG_E_INVAL, "triangle index out of range");
  for (long long i = 0; i < 2LL * nE; ++i)
    if (edges[i] < 0 || edges[i] >= nV) return fail(c, PNCG_E_INVAL, "edge index out of range");
  for (int e = 0; e < nE; ++e)
    if (edges[2 * e] == edges[2 * e + 1]) return fail(c, PNCG_E_INVAL, "degenerate edge");
  std::vector<double> Bm, vol;
  int bad = rest_shape(X, tets, nT, Bm, vol);
  if (bad >= 0) return fail(c, PNCG_E_INVERTED, "rest tet " + std::to_string(bad) + " has det <= 0");
  std::vector<int> inc, incv;
  if (!pack_incidence(nV, tets, nT, 0, inc, incv)) return fail(c, PNCG_E_INVAL, "a vertex belongs to more than 64 tets");
  // surface vertices and flags
  std::vector<uint8_t> fl(nV, 0);
  std::vector<int> surf;
  for (long long i = 0; i < 3LL * nF; ++i) fl[tris[i]] |= kSurface;
  for (int v = 0; v < nV; ++v)
    if (fl[v] & kSurface) surf.push_back(v);

  // commit host state
  c->nV = nV; c->nT = nT; c->nF = nF; c->nE = nE; c->nSV = (int)surf.size();
  c->X.assign(X, X + 3 * (size_t)nV);
  c->tets.assign(tets, tets + 4 * (size_t)nT);
  c->tris.assign(tris ? tris : tets, tris ? tris + 3 * (size_t)nF : tets);
  c->edges.assign(edges ? edges : tets, edges ? edges + 2 * (size_t)nE : tets);
  c->oid.assign(nV, 0);
  if (object_id) c->oid.assign(object_id, object_id + nV);
  c->surf = surf;
  c->vol = vol;
  c->Bm = Bm;
  c->vflag = fl;
  c->inc = inc;
  c->inc_vert = incv;
  c->nWaves = (int)(inc.size() / kWave);
  c->fixed.clear();
  c->fixed_target.clear();
  c->cflags = 0;
  c->planes.n = 0;
  c->kappa = 0.0;
  c->state = 1;
  c->grid = grid_for(c);

  int rc = ensure_device(c);
  if (rc) { c->state = 0; return rc; }
  HIPCHK(c, hipSetDevice(c->device));
  // (re)allocate device state
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  c->list_valid = false;
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  c->d_elem = nullptr; c->d_cand = nullptr; c->cand_cap = 0;
  c->d_cent = nullptr; c->d_cent_tmp = nullptr; c->d_ckey_tmp = nullptr;
  c->d_rp = nullptr;
  c->d_pv = nullptr;
  c->d_ovr = nullptr; c->n_ovr = 0; c->ovr_uploaded = false;
  c->ovr_set[0] = c->ovr_set[1] = false; c->ovr[0].clear(); c->ovr[1].clear();
  c->adj_ready = false; c->d_cgs = nullptr; c->cgs_cap = 0; c->E_uploaded = false;
  c->adj_lam_valid = false;
  c->d_excl_pt = c->d_excl_ee = nullptr; c->n_excl_pt = c->n_excl_ee = 0;
  const size_t r4 = (c->precision == PNCG_MIXED) ? sizeof(float4) : sizeof(double4);
  const int gmax = kMaxGrid;
  if ((rc = dmalloc(c, &c->d_inc, inc.size())) || (rc = dmalloc(c, &c->d_inc_vert, incv.size())) ||
      (rc = dmalloc(c, &c->d_mass, nV)) || (rc = dmalloc(c, &c->d_vflag, nV)) ||
      (rc = dmalloc(c, &c->d_target, nV)) || (rc = dmalloc(c, &c->d_x0, nV)) || (rc = dmalloc(c, &c->d_x1, nV)) ||
      (rc = dmalloc(c, &c->d_xbuild, nV)) ||
      (rc = dmalloc(c, &c->d_xt, nV)) || (rc = dmalloc(c, &c->d_xstart, nV)) ||
      (rc = dmalloc(c, (char**)&c->d_g, r4 * nV)) || (rc = dmalloc(c, (char**)&c->d_pg, r4 * nV)) ||
      (rc = dmalloc(c, (char**)&c->d_p0, r4 * nV)) || (rc = dmalloc(c, (char**)&c->d_p1, r4 * nV)) ||
      (rc = dmalloc(c, &c->d_acc, 8 * (size_t)nV)) || (rc = dmalloc(c, &c->d_tris, 3 * (size_t)nF)) ||
      (rc = dmalloc(c, &c->d_edges, 2 * (size_t)nE)) || (rc = dmalloc(c, &c->d_surf, surf.size())) ||
      (rc = dmalloc(c, &c->d_oid, nV)) || (rc = dmalloc(c, &c->d_ncand, 4)) ||
      (rc = dmalloc(c, &c->d_status, 1)) || (rc = dmalloc(c, &c->d_part_grad, 8 * (size_t)gmax)) ||
      (rc = dmalloc(c, &c->d_part_dir, 4 * (size_t)gmax)) || (rc = dmalloc(c, &c->d_part_narrow, gmax)) ||
      (rc = dmalloc(c, &c->d_io, 12 * (size_t)nV)) || (rc = dmalloc(c, &c->d_scalar, 8)) ||
      (rc = dmalloc(c, &c->d_item_lo, (size_t)nF + nE)) || (rc = dmalloc(c, &c->d_item_hi, (size_t)nF + nE)) ||
      (rc = dmalloc(c, &c->d_item_cnt, (size_t)nF + nE + surf.size())) ||
      (rc = dmalloc(c, &c->d_item_off, (size_t)nF + nE + surf.size() + 1)) ||
      (rc = dmalloc(c, &c->d_totals, 4)) ||
      (rc = dmalloc(c, &c->d_vcnt, 2 * (size_t)nV)) || (rc = dmalloc(c, &c->d_coff, (size_t)nV + 1)) ||
      (rc = dmalloc(c, &c->d_pl_tmp, (size_t)nV / kTileScan + 16)) || (rc = dmalloc(c, &c->d_big, (size_t)nV + 1)) || (rc = dmalloc(c, &c->d_wvert, (size_t)c->nWaves)) ||
      (rc = dmalloc(c, &c->d_wrange, (size_t)c->nWaves)))
    return rc;
  {
    // first and last vertex of every incidence wave (vertices ascend, padding at the end)
    std::vector<int2> wv(c->nWaves);
    for (int w = 0; w < c->nWaves; ++w) {
      int last = incv[(size_t)w * kWave];
      for (int l = 1; l < kWave; ++l) last = std::max(last, incv[(size_t)w * kWave + l]);
      wv[w] = make_int2(incv[(size_t)w * kWave], last);
    }
    HIPCHK(c, hipMemcpyAsync(c->d_wvert, wv.data(), sizeof(int2) * wv.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_wrange, 0, sizeof(int2) * wv.size(), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->scal_cap = 0;
  c->d_scal = nullptr;
  c->split_ready = false;
  c->oscal_cap = 0;
  c->d_oscal = nullptr;
  c->d_ent_key = nullptr; c->d_ent_item = nullptr; c->d_bkt_key = nullptr; c->d_bkt_item = nullptr;
  c->d_ent_rank = nullptr;
  c->d_bkt_lo = nullptr; c->d_bkt_hi = nullptr; c->d_bkt_ids = nullptr;
  c->d_count = nullptr; c->d_start = nullptr; c->d_part_cnt = nullptr; c->d_part_off = nullptr;
  // grid entries: start with eight cells per primitive; grown on demand
  if ((rc = alloc_grid(c, 8LL * (nF + nE) + (long long)surf.size() + 4096))) return rc;
  // the solver list's first capacity, so that steps start without allocating
  if ((rc = ensure_cand_cap(c, std::max<long long>(4096, 2LL * (long long)surf.size())))) return rc;
  HIPCHK(c, hipMemsetAsync(c->d_ncand, 0, 4 * sizeof(long long), c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_inc, inc.data(), sizeof(int) * inc.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_inc_vert, incv.data(), sizeof(int) * incv.size(), hipMemcpyHostToDevice, c->stream));
  if (nF) HIPCHK(c, hipMemcpyAsync(c->d_tris, tris, sizeof(int) * 3 * (size_t)nF, hipMemcpyHostToDevice, c->stream));
  if (nE) HIPCHK(c, hipMemcpyAsync(c->d_edges, edges, sizeof(int) * 2 * (size_t)nE, hipMemcpyHostToDevice, c->stream));
  if (!surf.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_surf, surf.data(), sizeof(int) * surf.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_oid, c->oid.data(), sizeof(int) * nV, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_acc, 0, sizeof(double) * 8 * (size_t)nV, c->stream));
  if ((rc = upload_flags_targets(c))) return rc;
  return sync(c);
}

int pncg_set_material(pncg_ctx* c, const double* E, const double* nu, const double* rho) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 1) return fail(c, PNCG_E_STATE, "set_mesh must come first");
  if (!E || !nu || !rho) return fail(c, PNCG_E_INVAL, "NULL material array");
  for (int e = 0; e < c->nT; ++e) {
    if (!std::isfinite(E[e]) || !std::isfinite(nu[e]) || !std::isfinite(rho[e]))
      return fail(c, PNCG_E_NONFINITE, "non-finite material parameter");
    if (!(E[e] > 0.0) || !(nu[e] >= 0.0 && nu[e] < 0.5) || !(rho[e] > 0.0))
      return fail(c, PNCG_E_INVAL, "material out of range (E > 0, 0 <= nu < 0.5, rho > 0)");
  }
  c->E.assign(E, E + c->nT);
  c->nu.assign(nu, nu + c->nT);
  c->rho.assign(rho, rho + c->nT);
  c->mass.assign(c->nV, 0.0);
  for (int e = 0; e < c->nT; ++e)
    for (int a = 0; a < 4; ++a) c->mass[c->tets[4 * e + a]] += rho[e] * c->vol[e] / 4.0;
  HIPCHK(c, hipSetDevice(c->device));
  int rc = (c->precision == PNCG_MIXED) ? upload_elements<float>(c) : upload_elements<double>(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->d_mass, c->mass.data(), sizeof(double) * c->nV, hipMemcpyHostToDevice, c->stream));
  c->E_uploaded = false;
  c->state = 2;
  return sync(c);
}

int pncg_set_contact(pncg_ctx* c, double dhat, double kappa, double cell, int32_t nP, const double* planes,
                     uint32_t flags) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 2) return fail(c, PNCG_E_STATE, "set_mesh and set_material must come first");
  if (!std::isfinite(dhat) || !std::isfinite(kappa) || !std::isfinite(cell) || !(dhat > 0.0) || kappa < 0.0 ||
      cell < 0.0)
    return fail(c, PNCG_E_INVAL, "need dhat > 0, kappa >= 0, cell >= 0");
  c->list_valid = false;
  if (nP < 0 || nP > kMaxPlanes || (nP > 0 && !planes)) return fail(c, PNCG_E_INVAL, "0 <= nP <= 8 planes");
  if (flags & ~3u) return fail(c, PNCG_E_INVAL, "unknown contact flag");
  Planes P{};
  P.n = nP;
  for (int j = 0; j < nP; ++j) {
    if (!finite_all(planes + 4 * j, 4)) return fail(c, PNCG_E_NONFINITE, "non-finite plane");
    const double n2 = planes[4 * j] * planes[4 * j] + planes[4 * j + 1] * planes[4 * j + 1] +
                      planes[4 * j + 2] * planes[4 * j + 2];
    if (std::fabs(std::sqrt(n2) - 1.0) > 1e-6) return fail(c, PNCG_E_INVAL, "plane normal must have unit length");
    for (int i = 0; i < 4; ++i) P.p[j][i] = planes[4 * j + i];
  }
  c->dhat = dhat;
  c->kappa = kappa;
  c->cell_user = cell;
  c->planes = P;
  c->cflags = flags;
  // grid cell: the caller's, or 1.5 x the mean rest length of the surface
  // edges (at least the candidate inflation), so each primitive touches a
  // few cells and a cell holds a few primitives
  double lsum = 0.0;
  for (int e = 0; e < c->nE; ++e) {
    const int a = c->edges[2 * e], b = c->edges[2 * e + 1];
    double l2 = 0.0;
    for (int i = 0; i < 3; ++i) l2 += (c->X[3 * a + i] - c->X[3 * b + i]) * (c->X[3 * a + i] - c->X[3 * b + i]);
    lsum += std::sqrt(l2);
  }
  const double lmean = c->nE > 0 ? lsum / c->nE : 0.0;
  c->lmean = lmean;
  c->skin = c->skin_user > 0.0 ? c->skin_user : default_skin(dhat, lmean);
  c->cell = cell > 0.0 ? cell : std::max(1.5 * lmean, dhat + c->skin);
  c->n_excl_pt = c->n_excl_ee = 0;
  HIPCHK(c, hipSetDevice(c->device));
  if ((flags & PNCG_CONTACT_SELF) && (flags & PNCG_CONTACT_REST_EXCLUDE) && c->nF + c->nE > 0) {
    // same-object pairs closer than 1.5 dhat in the rest shape (Sec. 5.1)
    int rc = stage_positions(c, c->X.data());
    if (rc) return rc;
    const double r = 1.5 * dhat;
    long long n = 0, npt = 0;
    if ((rc = build_candidates(c, c->d_x0, r, r, 1, &n, &npt))) return rc;
    std::vector<int2> pairs(n);
    if (n) HIPCHK(c, hipMemcpyAsync(pairs.data(), c->d_cand, sizeof(int2) * n, hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync(c))) return rc;
    std::vector<unsigned long long> kp, ke;
    for (long long i = 0; i < n; ++i) {
      const unsigned long long key = ((unsigned long long)(unsigned)pairs[i].x << 32) | (unsigned)pairs[i].y;
      (i < npt ? kp : ke).push_back(key);
    }
    std::sort(kp.begin(), kp.end());
    std::sort(ke.begin(), ke.end());
    if (!kp.empty()) {
      if ((rc = dmalloc(c, &c->d_excl_pt, kp.size()))) return rc;
      HIPCHK(c, hipMemcpyAsync(c->d_excl_pt, kp.data(), 8 * kp.size(), hipMemcpyHostToDevice, c->stream));
    }
    if (!ke.empty()) {
      if ((rc = dmalloc(c, &c->d_excl_ee, ke.size()))) return rc;
      HIPCHK(c, hipMemcpyAsync(c->d_excl_ee, ke.data(), 8 * ke.size(), hipMemcpyHostToDevice, c->stream));
    }
    c->n_excl_pt = (int)kp.size();
    c->n_excl_ee = (int)ke.size();
    if ((rc = sync(c))) return rc;
  }
  return PNCG_OK;
}

int pncg_set_solver(pncg_ctx* c, int32_t iter_max, double eps, int32_t term, const double* gravity, uint32_t flags) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 1) return fail(c, PNCG_E_STATE, "set_mesh must come first");
  if (iter_max < 1 || !std::isfinite(eps) || eps < 0.0 ||
      (term != PNCG_TERM_DELTA_E && term != PNCG_TERM_GRAD_REL && term != PNCG_TERM_GRAD_ABS))
    return fail(c, PNCG_E_INVAL, "need iter_max >= 1, eps >= 0, term DELTA_E, GRAD_REL or GRAD_ABS");
  if (gravity && !finite_all(gravity, 3)) return fail(c, PNCG_E_NONFINITE, "non-finite gravity");
  if ((flags & ~(3u | PNCG_BETA_MASK | PNCG_SPLIT_OBJECTS)) || (flags & PNCG_BETA_MASK) > PNCG_BETA_HZ)
    return fail(c, PNCG_E_INVAL, "unknown solver flag or beta rule");
  if (flags & PNCG_SPLIT_OBJECTS) {
    const char* why = split_layout_error(c);
    if (why) return fail(c, PNCG_E_INVAL, why);
  }
  c->iter_max = iter_max;
  c->eps = eps;
  c->term = term;
  if (gravity) for (int i = 0; i < 3; ++i) c->grav[i] = gravity[i];
  c->sflags = flags;
  return PNCG_OK;
}

int pncg_mean_boundary_edge(pncg_ctx* c, double* out) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 1) return fail(c, PNCG_E_STATE, "set_mesh must come first");
  if (!out) return fail(c, PNCG_E_INVAL, "NULL output");
  double lsum = 0.0;
  for (int e = 0; e < c->nE; ++e) {
    const int a = c->edges[2 * e], b = c->edges[2 * e + 1];
    double l2 = 0.0;
    for (int i = 0; i < 3; ++i) l2 += (c->X[3 * a + i] - c->X[3 * b + i]) * (c->X[3 * a + i] - c->X[3 * b + i]);
    lsum += std::sqrt(l2);
  }
  *out = c->nE > 0 ? lsum / c->nE : 0.0;
  return PNCG_OK;
}

int pncg_set_adjoint_warm_start(pncg_ctx* c, int32_t on) {
  if (!c) return PNCG_E_INVAL;
  if (on != 0 && on != 1) return fail(c, PNCG_E_INVAL, "on must be 0 or 1");
  c->adj_warm = on != 0;
  return PNCG_OK;
}

int pncg_set_model(pncg_ctx* c, int32_t model) {
  if (!c) return PNCG_E_INVAL;
  if (model < PNCG_MODEL_NH || model > PNCG_MODEL_FCR) return fail(c, PNCG_E_INVAL, "unknown material model");
  c->model = model;
  c->adj_lam_valid = false;
  if (c->state < 2) return PNCG_OK;
  HIPCHK(c, hipSetDevice(c->device));
  return (c->precision == PNCG_MIXED) ? upload_elements<float>(c) : upload_elements<double>(c);
}

int pncg_set_tuning(pncg_ctx* c, double skin, int32_t chunk) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 2) return fail(c, PNCG_E_STATE, "set_mesh and set_material must come first");
  if (!std::isfinite(skin) || skin < 0.0 || chunk < 0) return fail(c, PNCG_E_INVAL, "need skin >= 0, chunk >= 0");
  c->skin_user = skin;
  c->list_valid = false;
  c->skin = skin > 0.0 ? skin : default_skin(c->dhat, c->lmean);
  if (c->cell_user <= 0.0 && c->lmean > 0.0) c->cell = std::max(1.5 * c->lmean, c->dhat + c->skin);
  else if (c->cell_user <= 0.0) c->cell = c->dhat + c->skin;
  if (chunk > 0) c->chunk = chunk;
  return PNCG_OK;
}

int pncg_set_dirichlet(pncg_ctx* c, int32_t n, const int32_t* idx, const double* target) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 1) return fail(c, PNCG_E_STATE, "set_mesh must come first");
  if (n < 0 || (n > 0 && (!idx || !target))) return fail(c, PNCG_E_INVAL, "bad prescribed-vertex arrays");
  std::vector<char> seen(c->nV, 0);
  for (int i = 0; i < n; ++i) {
    if (idx[i] < 0 || idx[i] >= c->nV) return fail(c, PNCG_E_INVAL, "prescribed index out of range");
    if (seen[idx[i]]) return fail(c, PNCG_E_INVAL, "prescribed index repeated");
    seen[idx[i]] = 1;
  }
  if (n > 0 && !finite_all(target, 3 * (size_t)n)) return fail(c, PNCG_E_NONFINITE, "non-finite target");
  c->fixed.assign(idx, idx + n);
  c->fixed_target.assign(target, target + 3 * (size_t)n);
  HIPCHK(c, hipSetDevice(c->device));
  return upload_flags_targets(c);
}

// Object ranges and per-object buffers of the split step (allocated on the
// first split step after set_mesh; the per-iteration scalars grow with
// iter_max).
int pncg_set_candidates_override(pncg_ctx* c, int32_t kind, int64_t n, const int32_t* pairs) {
  if (!c) return PNCG_E_INVAL;
  if (c->state < 1) return fail(c, PNCG_E_STATE, "set_mesh must come first");
  c->list_valid = false;
  if (n < 0) {
    c->ovr_set[0] = c->ovr_set[1] = false;
    c->ovr[0].clear();
    c->ovr[1].clear();
    c->ovr_uploaded = false;
    return PNCG_OK;
  }
  if (kind != PNCG_KIND_PT && kind != PNCG_KIND_EE) return fail(c, PNCG_E_INVAL, "kind must be PNCG_KIND_PT or _EE");
  if (n > 0 && !pairs) return fail(c, PNCG_E_INVAL, "NULL pairs");
  if (n > (int64_t)INT_MAX / 8) return fail(c, PNCG_E_INVAL, "too many pairs");
  std::vector<int2> lst((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int a = pairs[2 * i], b = pairs[2 * i + 1];
    if (kind == PNCG_KIND_PT) {
      if (a < 0 || a >= c->nV || b < 0 || b >= c->nF)
        return fail(c, PNCG_E_INVAL, "point-triangle pair " + std::to_string(i) + " out of range");
      const int* t = c->tris.data() + 3 * (size_t)b;
      if (a == t[0] || a == t[1] || a == t[2])
        return fail(c, PNCG_E_INVAL, "point-triangle pair " + std::to_string(i) + " shares a vertex");
    } else {
      if (a < 0 || a >= c->nE || b < 0 || b >= c->nE || a == b)
        return fail(c, PNCG_E_INVAL, "edge-edge pair " + std::to_string(i) + " out of range or repeated edge");
      if (a > b) std::swap(a, b);
      const int* e1 = c->edges.data() + 2 * (size_t)a;
      const int* e2 = c->edges.data() + 2 * (size_t)b;
      if (e1[0] == e2[0] || e1[0] == e2[1] || e1[1] == e2[0] || e1[1] == e2[1])
        return fail(c, PNCG_E_INVAL, "edge-edge pair " + std::to_string(i) + " shares a vertex");
    }
    lst[(size_t)i] = make_int2(a, b);
  }
  std::vector<int2> srt(lst);
  std::sort(srt.begin(), srt.end(), [](const int2& p, const int2& q) { return p.x < q.x || (p.x == q.x && p.y < q.y); });
  for (size_t i = 1; i < srt.size(); ++i)
    if (srt[i].x == srt[i - 1].x && srt[i].y == srt[i - 1].y) return fail(c, PNCG_E_INVAL, "repeated pair");
  c->ovr[kind] = lst;
  c->ovr_set[kind] = true;
  c->ovr_uploaded = false;
  HIPCHK(c, hipSetDevice(c->device));
  int rc = upload_override(c);
  if (rc) return rc;
  if ((rc = ensure_cand_cap(c, std::max<long long>(c->n_ovr, 1024)))) return rc;
  return sync(c);
}

static int ensure_split(pncg_ctx* c) {
  if (!(c->sflags & PNCG_SPLIT_OBJECTS)) return PNCG_OK;
  int rc;
  if (!c->split_ready) {
    const char* why = split_layout_error(c);
    if (why) return fail(c, PNCG_E_INVAL, why);
    std::vector<int> vobj(c->nV), voff(1, 0), toff(1, 0);
    int n = 0;
    for (int v = 0; v < c->nV; ++v) {
      if (v > 0 && c->oid[v] != c->oid[v - 1]) { voff.push_back(v); ++n; }
      vobj[v] = n;
    }
    voff.push_back(c->nV);
    c->nObj = n + 1;
    for (int o = 0, e = 0; o < c->nObj; ++o) {
      while (e < c->nT && vobj[c->tets[4 * e]] == o) ++e;
      toff.push_back(e);
    }
    if ((rc = dmalloc(c, &c->d_vobj, c->nV)) || (rc = dmalloc(c, &c->d_voff, c->nObj + 1)) ||
        (rc = dmalloc(c, &c->d_toff, c->nObj + 1)) || (rc = dmalloc(c, &c->d_vdots, 6 * (size_t)c->nV)) ||
        (rc = dmalloc(c, &c->d_tphp, (size_t)c->nT)) || (rc = dmalloc(c, &c->d_vphp, 3 * (size_t)c->nV)) ||
        (rc = dmalloc(c, &c->d_opair, 2 * (size_t)c->nObj)))
      return rc;
    HIPCHK(c, hipMemcpyAsync(c->d_vobj, vobj.data(), sizeof(int) * c->nV, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_voff, voff.data(), sizeof(int) * voff.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_toff, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice, c->stream));
    c->split_ready = true;
  }
  if (c->oscal_cap < c->iter_max + 2) {
    if (c->d_oscal) dfree(c, c->d_oscal);
    c->d_oscal = nullptr;
    if ((rc = dmalloc(c, &c->d_oscal, (size_t)(c->iter_max + 2) * c->nObj))) return rc;
    c->oscal_cap = c->iter_max + 2;
    HIPCHK(c, hipMemsetAsync(c->d_oscal, 0, sizeof(ObjScal) * (size_t)c->oscal_cap * c->nObj, c->stream));
  }
  return sync(c);
}

static int ensure_scal(pncg_ctx* c) {
  if (c->scal_cap >= c->iter_max + 2) return PNCG_OK;
  if (c->d_scal) dfree(c, c->d_scal);
  c->d_scal = nullptr;
  int rc = dmalloc(c, &c->d_scal, (size_t)c->iter_max + 2);
  if (rc) return rc;
  c->scal_cap = c->iter_max + 2;
  HIPCHK(c, hipMemsetAsync(c->d_scal, 0, sizeof(IterScal) * c->scal_cap, c->stream));
  return PNCG_OK;
}

static int step_dev(pncg_ctx* c, const double* x, const double* v, double h, double* x_out, double* v_out,
                    pncg_stats* st, bool sync_end) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !v || !x_out || !v_out) return fail(c, PNCG_E_INVAL, "NULL state pointer");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = ensure_scal(c)) || (rc = ensure_split(c))) return rc;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (st) std::memset(st, 0, sizeof(*st));
    rc = c->precision == PNCG_MIXED ? step_impl<float>(c, x, v, h, x_out, v_out, st, sync_end)
                                    : step_impl<double>(c, x, v, h, x_out, v_out, st, sync_end);
    if (rc != kRestart) return rc;
    if ((rc = grow_solver_buffers(c))) return rc;
  }
  return fail(c, PNCG_E_CAPACITY, "candidate buffers kept overflowing");
}

int pncg_step_dev(pncg_ctx* c, const double* x, const double* v, double h, double* x_out, double* v_out,
                  pncg_stats* st) {
  return step_dev(c, x, v, h, x_out, v_out, st, true);
}

int pncg_step_dev_noalloc(pncg_ctx* c, const double* x, const double* v, double h, double* x_out, double* v_out,
                          pncg_stats* st) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !v || !x_out || !v_out) return fail(c, PNCG_E_INVAL, "NULL state pointer");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  if (c->iter_max > PNCG_NOALLOC_ITER_MAX)
    return fail(c, PNCG_E_INVAL, "iter_max above PNCG_NOALLOC_ITER_MAX (" + std::to_string(PNCG_NOALLOC_ITER_MAX) + ")");
  if (c->sflags & PNCG_SPLIT_OBJECTS) return fail(c, PNCG_E_INVAL, "the split step is not allocation-free");
  if (c->profiling) return fail(c, PNCG_E_STATE, "profiling is on (it creates events)");
  if (!c->d_static) return fail(c, PNCG_E_STATE, "no device scratch (set_mesh first)");
  if (c->grid > kMaxGrid) return fail(c, PNCG_E_INVAL, "grid above the scratch partials");
  HIPCHK(c, hipSetDevice(c->device));
  // the step's reduction scratch moves to this device's static array for the call
  unsigned char* base = static_cast<unsigned char*>(c->d_static);
  StepStatus* status = c->d_status;
  double *pg = c->d_part_grad, *pd = c->d_part_dir, *pn = c->d_part_narrow;
  IterScal* scal = c->d_scal;
  const int scal_cap = c->scal_cap;
  c->d_status = reinterpret_cast<StepStatus*>(base + kScratchStatus);
  c->d_part_grad = reinterpret_cast<double*>(base + kScratchPartGrad);
  c->d_part_dir = reinterpret_cast<double*>(base + kScratchPartDir);
  c->d_part_narrow = reinterpret_cast<double*>(base + kScratchPartNarrow);
  c->d_scal = reinterpret_cast<IterScal*>(base + kScratchScal);
  c->scal_cap = kScratchScalRecords;
  c->noalloc = true;
  if (st) std::memset(st, 0, sizeof(*st));
  rc = c->precision == PNCG_MIXED ? step_impl<float>(c, x, v, h, x_out, v_out, st)
                                  : step_impl<double>(c, x, v, h, x_out, v_out, st);
  c->noalloc = false;
  c->d_status = status;
  c->d_part_grad = pg;
  c->d_part_dir = pd;
  c->d_part_narrow = pn;
  c->d_scal = scal;
  c->scal_cap = scal_cap;
  if (rc == kRestart)
    return fail(c, PNCG_E_CAPACITY, "the contact buffers are too small for this state (a pncg_step_dev call grows them)");
  return rc;
}

int pncg_run_dev(pncg_ctx* c, double* x, double* v, double h, int32_t nsteps, pncg_stats* steps) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !v) return fail(c, PNCG_E_INVAL, "NULL state pointer");
  if (nsteps < 1) return fail(c, PNCG_E_INVAL, "need nsteps >= 1");
  int out = PNCG_OK;
  for (int i = 0; i < nsteps; ++i) {
    // in place: the predictor reads (x, v) before the step writes them; the
    // host waits for the end of the last step only
    rc = step_dev(c, x, v, h, x, v, steps ? steps + i : nullptr, i == nsteps - 1);
    if (rc < 0) return rc;
    out = std::max(out, rc);
  }
  return out;
}

int pncg_step(pncg_ctx* c, const double* x, const double* v, double h, double* x_out, double* v_out,
              pncg_stats* st) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !v || !x_out || !v_out) return fail(c, PNCG_E_INVAL, "NULL state pointer");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  const size_t n3 = 3 * (size_t)c->nV;
  if (!finite_all(x, n3) || !finite_all(v, n3)) return fail(c, PNCG_E_NONFINITE, "non-finite x or v");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = upload_rows(c, x, c->d_io, c->nV)) || (rc = upload_rows(c, v, c->d_io + n3, c->nV))) return rc;
  double* xo = c->d_io + 2 * n3;
  double* vo = c->d_io + 3 * n3;
  rc = pncg_step_dev(c, c->d_io, c->d_io + n3, h, xo, vo, st);
  if (rc < 0) return rc;
  HIPCHK(c, hipMemcpyAsync(x_out, xo, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(v_out, vo, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  int rs = sync(c);
  return rs ? rs : rc;
}

int pncg_energy(pncg_ctx* c, const double* x, const double* xt, double h, double* out) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !xt || !out) return fail(c, PNCG_E_INVAL, "NULL argument");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  HIPCHK(c, hipSetDevice(c->device));
  return c->precision == PNCG_MIXED ? energy_impl<float>(c, x, xt, h, out) : energy_impl<double>(c, x, xt, h, out);
}

int pncg_gradient(pncg_ctx* c, const double* x, const double* xt, double h, double* g, double* diag) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !xt || !g) return fail(c, PNCG_E_INVAL, "NULL argument");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  HIPCHK(c, hipSetDevice(c->device));
  return c->precision == PNCG_MIXED ? gradient_impl<float>(c, x, xt, h, g, diag)
                                    : gradient_impl<double>(c, x, xt, h, g, diag);
}

int pncg_hvp(pncg_ctx* c, const double* x, const double* p, double h, double* hp, double* php) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !p || !php) return fail(c, PNCG_E_INVAL, "NULL argument");
  if (!std::isfinite(h) || !(h > 0.0)) return fail(c, PNCG_E_INVAL, "need a finite h > 0");
  HIPCHK(c, hipSetDevice(c->device));
  return c->precision == PNCG_MIXED ? hvp_impl<float>(c, x, p, h, hp, php) : hvp_impl<double>(c, x, p, h, hp, php);
}

int pncg_candidates(pncg_ctx* c, const double* x, int32_t kind, int32_t* pairs, int64_t cap, int64_t* n) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !n || cap < 0 || (cap > 0 && !pairs)) return fail(c, PNCG_E_INVAL, "bad arguments");
  if (kind < PNCG_KIND_PT || kind > PNCG_KIND_PG) return fail(c, PNCG_E_INVAL, "unknown kind");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = stage_positions(c, x))) return rc;
  std::vector<int2> out;
  if (kind == PNCG_KIND_PG) {
    const long long capd = (long long)c->nSV * std::max(c->planes.n, 1);
    if (capd > c->cand_cap && (rc = ensure_cand_cap(c, std::max<long long>(capd, 1024)))) return rc;
    Broad B = make_broad(c);
    plane_candidates(B, c->d_x0, c->planes, c->dhat, c->d_cand, c->d_ncand, c->cand_cap, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->h_n, c->d_ncand, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync(c))) return rc;
    const long long m = c->h_n[0];
    out.resize(m);
    if (m) HIPCHK(c, hipMemcpyAsync(out.data(), c->d_cand, sizeof(int2) * m, hipMemcpyDeviceToHost, c->stream));
  } else if ((c->cflags & PNCG_CONTACT_SELF) && c->nF + c->nE > 0) {
    long long m = 0, mpt = 0;
    if ((rc = build_candidates(c, c->d_x0, c->dhat, -1.0, 0, &m, &mpt))) return rc;
    const long long a = kind == PNCG_KIND_PT ? 0 : mpt, b = kind == PNCG_KIND_PT ? mpt : m;
    out.resize(b - a);
    if (b > a) HIPCHK(c, hipMemcpyAsync(out.data(), c->d_cand + a, sizeof(int2) * (b - a), hipMemcpyDeviceToHost, c->stream));
  }
  if ((rc = sync(c))) return rc;
  std::sort(out.begin(), out.end(), [](const int2& p, const int2& q) { return p.x < q.x || (p.x == q.x && p.y < q.y); });
  *n = (int64_t)out.size();
  if ((int64_t)out.size() > cap) return fail(c, PNCG_E_CAPACITY, "pairs buffer too small; *n holds the size needed");
  for (size_t i = 0; i < out.size(); ++i) {
    pairs[2 * i] = out[i].x;
    pairs[2 * i + 1] = out[i].y;
  }
  return PNCG_OK;
}

int pncg_solver_pairs(pncg_ctx* c, const double* x, int32_t kind, int32_t* pairs, int64_t cap, int64_t* n) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !n || cap < 0 || (cap > 0 && !pairs)) return fail(c, PNCG_E_INVAL, "bad arguments");
  if (kind != PNCG_KIND_PT && kind != PNCG_KIND_EE) return fail(c, PNCG_E_INVAL, "kind must be PNCG_KIND_PT or _EE");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = stage_positions(c, x))) return rc;
  c->list_valid = false;
  std::vector<int2> all;
  if ((c->cflags & PNCG_CONTACT_SELF) && c->nF + c->nE > 0) {
    if ((rc = ensure_cand_cap(c, std::max<long long>(4096, 2LL * c->nSV)))) return rc;
    long long cnt[2] = {0, 0};
    for (int attempt = 0;; ++attempt) {
      broad_solver_list(make_broad(c), c->d_x0, c->cell, c->dhat + c->skin, c->d_cand, c->cand_cap, c->d_ncand,
                        &c->d_status->err, &c->d_status->n_cand, c->stream);
      HIPCHK(c, hipMemcpyAsync(&cnt[0], c->d_totals, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(&cnt[1], c->d_ncand, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
      if ((rc = sync(c))) return rc;
      if (cnt[0] <= c->ent_cap && cnt[1] <= c->cand_cap) break;
      if (attempt == 2) return fail(c, PNCG_E_NOMEM, "the solver's list did not fit after growing its buffers");
      if (cnt[0] > c->ent_cap && (rc = alloc_grid(c, cnt[0] + cnt[0] / 2))) return rc;
      if (cnt[1] > c->cand_cap && (rc = ensure_cand_cap(c, cnt[1] + cnt[1] / 2 + 1024))) return rc;
    }
    all.resize((size_t)cnt[1]);
    if (cnt[1]) HIPCHK(c, hipMemcpyAsync(all.data(), c->d_cand, sizeof(int2) * cnt[1], hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync(c))) return rc;
  }
  // the kind is in the pair: (v, f) point-triangle, (e1, ~e2) edge-edge
  std::vector<int2> out;
  for (const int2& p : all) {
    if (kind == PNCG_KIND_PT && p.y >= 0) out.push_back(p);
    if (kind == PNCG_KIND_EE && p.y < 0) out.push_back(make_int2(p.x, ~p.y));
  }
  std::sort(out.begin(), out.end(), [](const int2& p, const int2& q) { return p.x < q.x || (p.x == q.x && p.y < q.y); });
  *n = (int64_t)out.size();
  if ((int64_t)out.size() > cap) return fail(c, PNCG_E_CAPACITY, "pairs buffer too small; *n holds the size needed");
  for (size_t i = 0; i < out.size(); ++i) {
    pairs[2 * i] = out[i].x;
    pairs[2 * i + 1] = out[i].y;
  }
  return PNCG_OK;
}

int pncg_set_profiling(pncg_ctx* c, int32_t on) {
  if (!c) return PNCG_E_INVAL;
  c->profiling = on != 0;
  for (int i = 0; i < PNCG_PROF_KINDS; ++i) {
    c->prof_us[i] = 0.0;
    c->prof_n[i] = 0;
  }
  c->ev_pending.clear();
  c->ev_used = 0;
  return PNCG_OK;
}

int pncg_get_profile(pncg_ctx* c, double* total_us, int64_t* launches) {
  if (!c || !total_us || !launches) return PNCG_E_INVAL;
  for (int i = 0; i < PNCG_PROF_KINDS; ++i) {
    total_us[i] = c->prof_us[i];
    launches[i] = c->prof_n[i];
  }
  return PNCG_OK;
}

int pncg_min_distance(pncg_ctx* c, const double* x, double* dmin, double* jmin) {
  int rc = ready(c);
  if (rc) return rc;
  if (!x || !dmin || !jmin) return fail(c, PNCG_E_INVAL, "NULL argument");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = stage_positions(c, x))) return rc;
  const bool self = (c->cflags & PNCG_CONTACT_SELF) && c->nF + c->nE > 0;
  if (self) {
    if ((rc = build_candidates(c, c->d_x0, 10.0 * c->dhat, -1.0, 0, nullptr, nullptr))) return rc;
  } else {
    HIPCHK(c, hipMemsetAsync(c->d_ncand, 0, 2 * sizeof(long long), c->stream));
  }
  std::vector<double> part(2 * (size_t)c->grid);
  if (c->precision == PNCG_MIXED) {
    Args<float> A = make_args<float>(c, 1.0);
    A.self = self;
    launch_audit<float>(A, c->d_part_dir, c->stream);
  } else {
    Args<double> A = make_args<double>(c, 1.0);
    A.self = self;
    launch_audit<double>(A, c->d_part_dir, c->stream);
  }
  HIPCHK(c, hipMemcpyAsync(part.data(), c->d_part_dir, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
  if ((rc = sync(c))) return rc;
  double d = HUGE_VAL, j = HUGE_VAL;
  for (int b = 0; b < c->grid; ++b) {
    d = std::min(d, part[2 * b]);
    j = std::min(j, part[2 * b + 1]);
  }
  *dmin = d;
  *jmin = j;
  return PNCG_OK;
}


int pncg_adjoint_step_dev(pncg_ctx* c, const double* x1, double h, const double* xbar, const double* vbar,
                          double cg_tol, int32_t cg_max, double* xbar_t, double* vbar_t, double* Ebar,
                          pncg_adjoint_stats* st) {
  int rc = adjoint_checks(c, x1, h, xbar, vbar, cg_tol, cg_max, xbar_t, vbar_t, Ebar);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  if (st) std::memset(st, 0, sizeof(*st));
  return adjoint_impl(c, x1, h, xbar, vbar, cg_tol, cg_max, xbar_t, vbar_t, Ebar, st);
}

int pncg_adjoint_step(pncg_ctx* c, const double* x1, double h, const double* xbar, const double* vbar,
                      double cg_tol, int32_t cg_max, double* xbar_t, double* vbar_t, double* Ebar,
                      pncg_adjoint_stats* st) {
  int rc = adjoint_checks(c, x1, h, xbar, vbar, cg_tol, cg_max, xbar_t, vbar_t, Ebar);
  if (rc) return rc;
  const size_t n3 = 3 * (size_t)c->nV;
  if (!finite_all(x1, n3) || !finite_all(xbar, n3) || !finite_all(vbar, n3) || !finite_all(Ebar, c->nT))
    return fail(c, PNCG_E_NONFINITE, "non-finite input");
  HIPCHK(c, hipSetDevice(c->device));
  if ((rc = ensure_adjoint(c, cg_max))) return rc;
  if (st) std::memset(st, 0, sizeof(*st));
  // inputs in d_io (x1, xbar, vbar), outputs in d_aio (xbar_t, vbar_t, Ebar)
  double* dx = c->d_io;
  double* dxb = c->d_io + n3;
  double* dvb = c->d_io + 2 * n3;
  double* oxb = c->d_aio;
  double* ovb = c->d_aio + n3;
  double* oE = c->d_aio + 2 * n3;
  if ((rc = upload_rows(c, x1, dx, c->nV)) || (rc = upload_rows(c, xbar, dxb, c->nV)) ||
      (rc = upload_rows(c, vbar, dvb, c->nV)))
    return rc;
  HIPCHK(c, hipMemcpyAsync(oE, Ebar, sizeof(double) * c->nT, hipMemcpyHostToDevice, c->stream));
  rc = adjoint_impl(c, dx, h, dxb, dvb, cg_tol, cg_max, oxb, ovb, oE, st);
  if (rc < 0) return rc;
  HIPCHK(c, hipMemcpyAsync(xbar_t, oxb, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(vbar_t, ovb, sizeof(double) * n3, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(Ebar, oE, sizeof(double) * c->nT, hipMemcpyDeviceToHost, c->stream));
  int rs = sync(c);
  return rs ? rs : rc;
}

}  // extern "C"
