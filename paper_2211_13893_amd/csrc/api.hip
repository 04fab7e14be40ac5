// C ABI entry points: plans, assembly, the LOBPCG driver and operator application.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.hpp"
#include "msgfem.h"

namespace msg {
__global__ void k_materials(const double*, int, double*);
__global__ void k_pou_total(const int32_t*, int, int, int, int, int, int32_t*);
__global__ void k_fill_i32(int32_t*, int64_t, int32_t);
__global__ void k_fill_f64(double*, int64_t, double);
__global__ void k_assemble(const BoxMeta*, MeshDev, const double*, double*);
__global__ void k_classes_mu(const BoxMeta*, MeshDev, int, const int32_t*, uint8_t*, double*);
__global__ void k_band_build(const BoxMeta*, int, const double*, const uint8_t*, const double*, double,
                             double*);
__global__ void k_chol_update(const MatDesc*, int, double*, int32_t*);
__global__ void k_chol_panel(const MatDesc*, int, double*);
template <int P>
__global__ void k_chol_step(const MatDesc*, int, int, int, int, double*, int32_t*);
template <int P>
__global__ void k_chol_matrix(const MatDesc*, int, double*, int32_t*);
#define CHOL_PANEL 4   // panel columns of the tile Cholesky (k_chol_step<P>)
__global__ void k_chol_unit(const MatDesc*, double*);
__global__ void k_band_unit_relayout4(const BoxMeta*, int, double*, int);
__global__ void k_band_relayout(const BoxMeta*, int, double*);
__global__ void k_band_relayout4(const BoxMeta*, int, double*, int);
template <int KC, int NS, typename T>
__global__ void k_band_solve(const BoxMeta*, int, int, int, const T*, const uint8_t*, const double*, double*, int,
                             int, int, double*, int64_t, const int32_t*, int, double*, int64_t, const int32_t*);
template <int NSLOT, bool WIDE, typename T>
__global__ void k_band_solve4(const BoxMeta*, int, int, int, const T*, const uint8_t*, const double*, double*, int,
                              int, int, double*, int64_t, const int32_t*, int, double*, int64_t, const int32_t*);
__global__ void k_sep_syrk(const SepDesc*, int, int, double*);

template <bool TWO, int CW, typename ST>
__global__ void k_spmm(const BoxMeta*, int, int, const ST*, const uint8_t*, const double*, const double*,
                       double*, double*, int, int, double, const int32_t*);
template <bool TWO, typename ST>
__global__ void k_spmm_planes(const BoxMeta*, int, int, int, const ST*, const uint8_t*, const double*,
                              const double*, double*, double*, int, int, double, const int32_t*);
#define SP_PLANE 240   // nodes of a staged plane tile (k_spmm_planes)
static int sp_tile_x_host(int mx, int my) {
  if (mx * my <= SP_PLANE) return mx;
  const int t = SP_PLANE / my - 2;
  return t >= 1 ? t : 0;
}
static size_t sp_lds(bool two) { return (size_t)3 * 3 * SP_PLANE * 4 * 16 + (two ? (size_t)3 * 3 * SP_PLANE * 8 : 0); }
__global__ void k_mixed_copies(const BoxMeta*, int, const double*, float*, const double*, float*);
__global__ void k_mask_b3(const uint8_t*, const double*, int, int64_t, double*);
__global__ void k_keep_classes(const uint8_t*, int, int, int64_t, double*);
struct Blk3 { const double* p[3]; };
struct Blk4x3 { const double* p[4][3]; };
struct Out4 { double* p[4]; };
template <int NB>
__global__ void k_gram_partial(const BoxMeta*, int, Blk3, Blk3, Blk3, int, int, int, double*,
                               const int32_t*);
__global__ void k_gram_reduce(int, int, const double*, double*, const int32_t*);
__global__ void k_rayleigh_ritz(int, int, int, double, const double*, double*, double*, double*,
                                double*, const int32_t*);
template <int CB>
__global__ void k_update(const BoxMeta*, int, int, Blk4x3, Out4, Out4, const double*, const double*,
                         const int32_t*);
__global__ void k_proj_coef(int, double, const double*, double*, const int32_t*);
__global__ void k_keep_cols(const BoxMeta*, int, int, int, XLoc, int, double*);
__global__ void k_residual(const BoxMeta*, const uint8_t*, int, int, double, const double*, const double*,
                           const double*, double*, int, int, double*, const int32_t*);
__global__ void k_converge(const BoxMeta*, int, int, int, const double*, const double*, double, double, double*,
                           int32_t*, int32_t*, int32_t*, int, int32_t*, int, int, const int32_t*, int32_t*, int,
                           int32_t*);
__global__ void k_add_i32(int32_t*, int32_t);
__global__ void k_status_clear(int, const int32_t*, int32_t*);
__global__ void k_status_or(int32_t*, int, int32_t);
__global__ void k_copy_masked_i32(int, const int32_t*, const int32_t*, int32_t*);
__global__ void k_random_start(const BoxMeta*, const uint8_t*, int, int, uint64_t, double*);
__global__ void k_lock(const BoxMeta*, int, const double*, double, double*, double*, double*, double*, double*,
                       const int32_t*);
__global__ void k_copy_start(const BoxMeta*, const uint8_t*, int, int, const double*, double*);
__global__ void k_output(const BoxMeta*, int, double, XLoc, const double*, const double*,
                         double*, double*, double*, const int32_t*, int, int);
struct FaceLoad {
  int32_t axis, side;
  double g[3];
};
struct CoarsePair {
  int32_t i, j;
  int32_t lo[3], hi[3];
  int32_t row_off, col_off;
};
__global__ void k_box_load(const BoxMeta*, MeshDev, const FaceLoad*, int, double*);
__global__ void k_coarse_basis(const BoxMeta*, int, const double*, const double*, const double*, double*,
                               double*);
__global__ void k_cholqr_coef(int, const double*, double*);
__global__ void k_select_modes(const BoxMeta*, const double*, double, const double*, double*, int32_t*, int32_t*);
__global__ void k_error_norms(MeshDev, const double*, const double*, double*);
__global__ void k_box_digest(const BoxMeta*, const double*, const double*, const uint8_t*, unsigned long long*);
__global__ void k_box_digest_finish(const BoxMeta*, int, uint64_t, unsigned long long*);
__global__ void k_copy_eigs(int, int64_t, const double*, const double*, const double*, const int32_t*, double*,
                            double*, double*, int32_t*);
__global__ void k_coarse_pairs(const BoxMeta*, const CoarsePair*, int, const double*, const double*,
                               const double*, int, int, double*, double*);
__global__ void k_coarse_rhs(const BoxMeta*, int, const double*, const double*, const int32_t*,
                             const int32_t*, int, int, const double*, double*, double*);
__global__ void k_dense_tiles(const double*, int, int, double*);
__global__ void k_trsv_init(const double*, int, int, double*);
__global__ void k_trsv_fwd(const double*, int, int, double*);
__global__ void k_trsv_diag(const double*, int, const double*, double*);
__global__ void k_trsv_bwd(const double*, int, int, double*);
__global__ void k_store_box(const BoxMeta*, const BoxMeta*, int, int, const double*, const double*, const double*,
                            const double*, const double*, const uint8_t*, double*, double*, double*, double*,
                            double*, uint8_t*);
__global__ void k_store_local32(const BoxMeta*, const BoxMeta*, const double*, float*);
__global__ void k_prolong(const BoxMeta*, MeshDev, int, const double*, const double*, const double*,
                          const int32_t*, double*, double*);
__global__ void k_gather_boxes(const BoxMeta*, MeshDev, const uint8_t*, const double*, double*);
__global__ void k_scatter_boxes(const BoxMeta*, MeshDev, const uint8_t*, const double*, double*);
__global__ void k_coarse_restrict(const BoxMeta*, int, const double*, const double*, const int32_t*, double*);
__global__ void k_dot_partial(const double*, const double*, const uint8_t*, int64_t, double*);
__global__ void k_dot_final(const double*, int, double*);
__global__ void k_pcg_alpha(double*);
__global__ void k_pcg_beta(double*);
__global__ void k_pcg_xr(const uint8_t*, int64_t, const double*, const double*, const double*, double*,
                         double*);
__global__ void k_pcg_p(const uint8_t*, int64_t, const double*, const double*, double*);
__global__ void k_sub(const uint8_t*, int64_t, const double*, const double*, double*);
__global__ void k_warm_features(const BoxMeta*, MeshDev, float*);
__global__ void k_warm_basis(const BoxMeta*, const uint8_t*, const double*, int, int, double*);
__global__ void k_warm_labels(const BoxMeta*, const uint8_t*, const double*, const double*, int, int, float*);
__global__ void k_warm_start(const BoxMeta*, const uint8_t*, const float*, const double*, int, int, int, uint64_t,
                             double*);
}  // namespace msg

using namespace msg;

static const int KC = 8;           // columns per solve workgroup (16 in the wide matrix-core solve)
// the wide matrix-core solve (16 columns per workgroup, v_mfma_f64_16x16x4f64)
// keeps a ring of BT rows x 16 columns and 8 x 32 x 17 partial sums in LDS:
// bands of at most 31 tiles
static const int WIDE_MAX_BT = 31;
// eigenpairs per box: beyond 32 they come in deflated rounds; two rounds at
// most, because a third round's pairs can sit 1e4 below the first round's in
// nu (the end subdomains of a clamped beam), where the first round's error is
// amplified past what the FP64 images resolve
static const int MAX_NEV = 48;
static const int ROUND_PAIRS = 24; // pairs per deflated round (block 32, 8 guard columns)
static const int GRAM_ROWS = 1024; // rows per Gram / residual chunk

// the Gram partials of every (row chunk, box): 64 threads per 16-column
// block of the m columns (m <= 96), both products from one workgroup
static void gram_partials(int m, int n_chunk, int nb, hipStream_t s, const BoxMeta* meta, int nblk, Blk3 Z,
                          Blk3 A, Blk3 B, int k, double* part, const int32_t* act) {
  const int nb16 = (m + 15) / 16;
  const dim3 grid(n_chunk, nb);
  if (nb16 <= 2)
    k_gram_partial<2><<<grid, 128, 0, s>>>(meta, nblk, Z, A, B, k, GRAM_ROWS, n_chunk, part, act);
  else if (nb16 <= 4)
    k_gram_partial<4><<<grid, 256, 0, s>>>(meta, nblk, Z, A, B, k, GRAM_ROWS, n_chunk, part, act);
  else
    k_gram_partial<6><<<grid, 384, 0, s>>>(meta, nblk, Z, A, B, k, GRAM_ROWS, n_chunk, part, act);
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }
// dynamic LDS of k_update<cb> for an m x k coefficient pair staged in
// operand order (groups of 64 doubles per 4 inner indices and 16 columns)
static size_t upd_lds(int m, int cb) { return (size_t)2 * ((m + 7) / 8) * 2 * cb * 64 * 8; }

struct msgfem_plan {
  int device = 0;
  msgfem_mesh mesh{};
  int32_t nsd = 0, overlap = 0;
  std::vector<int32_t> omega;     // [nsd][6] node boxes of Omega_j
  std::vector<BoxMeta> meta;      // batch boxes
  std::vector<MatDesc> mats;      // the two banded matrices of every box (A11, Ahat)
  msgfem_eig_opts opts{};
  int k = 0;
  int nround = 0;    // eigenpairs per deflated round (n_ev > 32 takes several rounds)
  int rounds = 1;
  int kv = 0;        // columns of a coarse basis block (max(k, max n_ev) rounded up to 8)
  int64_t n_nodes_global = 0;
  // ops layout (bytes)
  int64_t o_meta = 0, o_mats = 0, o_omega = 0, o_ctab = 0, o_wtot = 0, o_stencil = 0, o_mu = 0,
          o_cls = 0, o_fac = 0, o_fac32 = 0, o_st32 = 0, ops_bytes = 0;
  int64_t nodes_total = 0, dofs_total = 0, fac_total = 0, vec_total = 0, evec_total = 0,
          eval_total = 0;
  int max_nodes = 0, max_dof = 0, max_nt = 0, max_bt = 0;
  int max_bt_kind[2] = {0, 0};   // per matrix kind (A11, Ahat)
  int64_t max_fac_tiles = 0;
  // nested dissection of the box matrices (MSGFEM_OPT_SPLIT)
  int split = 1;
  int solve_pref = 0;            // MSGFEM_OPT_SOLVE
  int spmm_pref = 0;             // MSGFEM_OPT_SPMM
  int chol_pref = 0;             // MSGFEM_OPT_CHOL
  int n_cu = 0;                  // compute units of the device (read at the first factorisation; -1: unknown)
  bool any_split[2] = {false, false};
  int max_nts = 0;               // separator tile rows
  int n_chain_mats = 0;          // mats[0 .. n_chain_mats): whole bands and chains; then the separator blocks
  std::vector<SepDesc> seps;
  int64_t o_seps = 0, w_sep = 0, sep_q = 0;
  std::vector<int32_t> order;    // [kind][nb]: batch boxes by decreasing block-solve sweep length
  int64_t o_order = 0;
  int n_gchunk = 0;
  // work layout (bytes)
  int64_t w_vec = 0, w_part = 0, w_G = 0, w_L = 0, w_Y = 0, w_Yp = 0, w_nu = 0, w_rho = 0,
          w_rpart = 0, w_active = 0, w_iters = 0, w_nact = 0, w_reached = 0, w_xbuf = 0, w_scr = 0,
          work_bytes = 0;
  int64_t scr_stride = 0;
  // coarse problem (built on the first coarse call)
  bool coarse_ready = false;
  int NH = 0, NTc = 0;
  std::vector<CoarsePair> pairs;
  std::vector<int32_t> pair_start, row_off;
  int64_t c_faces = 0, c_pairs = 0, c_pstart = 0, c_roff = 0, c_mat = 0, c_bload = 0, c_psi = 0,
          c_pv = 0, c_V = 0, c_Vn = 0, c_AV = 0, c_Ap = 0, c_rpart = 0, c_tiles = 0, c_y = 0,
          coarse_bytes = 0;
  std::string err;
  // kernel timing (msgfem_profile)
  struct ProfRec {
    int kernel;
    hipEvent_t b, e;
    double bytes, flops;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[16] = {}, prof_bytes[16] = {}, prof_flops[16] = {};
  int64_t prof_launches[16] = {};
  // LOBPCG iterations captured in HIP graphs (msgfem_plan_set_option)
  int graph_mode = 0;
  hipStream_t cap_stream = nullptr;   // capture only: the graphs are launched on the caller's stream
  struct GraphEntry {
    const void* ops;
    const void* work;
    const int32_t* status;
    int r, pre32;
    double lock_tol;
    double* B[4][5];
    int L;                            // iterations per launch
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int64_t graph_launches = 0;         // graph launches of the last msgfem_local_eigs call
  int64_t graph_iters = 0;            // LOBPCG iterations they ran
  ~msgfem_plan();
};

static const char* const PROF_NAMES[] = {"assemble", "band_build", "band_potrf", "band_solve",
                                         "spmm", "gram", "rayleigh_ritz", "update", "residual"};
enum { PK_ASSEMBLE, PK_BUILD, PK_POTRF, PK_SOLVE, PK_SPMM, PK_GRAM, PK_RR, PK_UPDATE, PK_RESID, PK_N };

msgfem_plan::~msgfem_plan() {
  for (auto& r : prof_pending) { ev_pool.push_back(r.b); ev_pool.push_back(r.e); }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

static hipEvent_t prof_event(msgfem_plan* p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records HIP events around one launch on the launch stream when profiling is on.
struct ProfScope {
  msgfem_plan* p;
  int kernel;
  hipStream_t s;
  hipEvent_t b = nullptr;
  double bytes, flops;
  bool on;
  ProfScope(msgfem_plan* p_, int kernel_, hipStream_t s_, double bytes_, double flops_, bool allow = true)
      : p(p_), kernel(kernel_), s(s_), bytes(bytes_), flops(flops_), on(allow && p_->prof_on) {
    if (on) {
      b = prof_event(p);
      if (b) (void)hipEventRecord(b, s);
    }
  }
  ~ProfScope() {
    if (on && b) {
      hipEvent_t e = prof_event(p);
      if (e) {
        (void)hipEventRecord(e, s);
        p->prof_pending.push_back({kernel, b, e, bytes, flops});
      }
    }
  }
};

static int fail(msgfem_plan* p, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (p) p->err = buf;
  return code;
}

#define HIPCHK(p, call)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(p, MSGFEM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

#define LAUNCHCHK(p)                                                                       \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess)                                                                  \
      return fail(p, MSGFEM_EHIP, "launch failed (line %d): %s", __LINE__,                 \
                  hipGetErrorString(e_));                                                  \
  } while (0)

// Band of the lexicographic node order of a (sub-)box with node dims d[3]:
// the order runs over the box axes from the shortest (fastest index) to the
// longest (slowest), which minimises the half-bandwidth 3 (s0 s1 + s0 + 1) + 2
// (ties keep the axis order x, y, z).  ord encodes the axes (BoxMeta.ord).
static void band_geom(const int d[3], int* n, int* nt, int* bt, int32_t* ord) {
  int a[3] = {0, 1, 2};
  std::stable_sort(a, a + 3, [&](int x, int y) { return d[x] < d[y]; });
  const int s0 = d[a[0]], s1 = d[a[1]];
  *ord = a[0] | (a[1] << 2) | (a[2] << 4);
  *n = 3 * d[0] * d[1] * d[2];
  int b = 3 * (s0 * s1 + s0 + 1) + 2;
  *nt = (*n + 31) / 32;
  *bt = (b + 31) / 32 + 1;
  if (*bt > *nt) *bt = *nt;
}

// Geometry of the box of subdomain sd (Omega_j^*, or Omega_j for GenEO): node
// box, Omega_j, interior-face flags, the node sub-box of B1 and the band
// geometry of its two matrices.  Offsets are left zero.  omega: [nsd][6] node
// boxes of Omega_j.  Returns an error message or nullptr.
static const char* box_geometry(const int N[3], const msgfem_decomp* dec, const int32_t* omega, bool geneo, int sd,
                                int n_ev, BoxMeta& m) {
  std::memset(&m, 0, sizeof m);
  m.sd = sd;
  const int32_t* c = dec->cores + 6 * sd;
  int g = dec->overlap + (geneo ? 0 : dec->ovs[sd]);   // GenEO works on Omega_j itself
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = std::max(c[d] - g, 0);
    hi[d] = std::min(c[3 + d] + g, N[d]);
    m.g0[d] = lo[d];
    m.olo[d] = omega[6 * sd + d];
    m.ohi[d] = omega[6 * sd + 3 + d];
    m.olo_int[d] = m.olo[d] > 0;
    m.ohi_int[d] = m.ohi[d] < N[d];
    m.iface_lo[d] = lo[d] > 0;
    m.iface_hi[d] = hi[d] < N[d];
  }
  m.mx = hi[0] - lo[0] + 1;
  m.my = hi[1] - lo[1] + 1;
  m.mz = hi[2] - lo[2] + 1;
  int mm[3] = {m.mx, m.my, m.mz};
  for (int d = 0; d < 3; ++d) {
    m.sub_lo[d] = m.iface_lo[d] ? 1 : 0;
    m.sub_hi[d] = mm[d] - 1 - (m.iface_hi[d] ? 1 : 0);
    if (m.sub_hi[d] < m.sub_lo[d] || mm[d] < 3) return "box too thin for an interior block";
  }
  if (!(m.iface_lo[0] || m.iface_hi[0] || m.iface_lo[1] || m.iface_hi[1] || m.iface_lo[2] || m.iface_hi[2]))
    return "oversampling box covers the whole mesh (B2 empty)";
  m.n_nodes = m.mx * m.my * m.mz;
  m.n_dof = 3 * m.n_nodes;
  m.n_ev = n_ev;
  const int d11[3] = {m.sub_hi[0] - m.sub_lo[0] + 1, m.sub_hi[1] - m.sub_lo[1] + 1, m.sub_hi[2] - m.sub_lo[2] + 1};
  band_geom(d11, &m.n11, &m.nt11, &m.bt11, &m.ord[0]);
  band_geom(mm, &m.nh, &m.nth, &m.bth, &m.ord[1]);
  return nullptr;
}

// Nested dissection of a box matrix: split when its slowest order axis has
// at least this many node layers (each chain then has at least 3.5 layers)
static const int SPLIT_MIN_LAYERS = 8;

// The band parts of both box matrices (geometry only; offsets in plan_layout):
// one whole band, or with split two chains of (layers before / after the
// middle layer zs) + separator rows and the separator block.
static void band_parts(BoxMeta& m, bool split) {
  for (int kind = 0; kind < 2; ++kind) {
    int d[3];
    for (int a = 0; a < 3; ++a)
      d[a] = kind == 0 ? m.sub_hi[a] - m.sub_lo[a] + 1 : (a == 0 ? m.mx : (a == 1 ? m.my : m.mz));
    const int ord = m.ord[kind];
    const int s0 = d[ord & 3], s1 = d[(ord >> 2) & 3], s2 = d[(ord >> 4) & 3];
    const int n = kind ? m.nh : m.n11, NT = kind ? m.nth : m.nt11, BT = kind ? m.bth : m.bt11;
    BandPart* q = m.part[kind];
    for (int pi = 0; pi < 3; ++pi) q[pi] = BandPart{};
    m.nd[kind] = 0;
    m.zs[kind] = 0;
    if (split && s2 >= SPLIT_MIN_LAYERS) {
      const int L = 3 * s0 * s1, zs = s2 / 2;
      const int n0 = L * zs, n1 = L * (s2 - zs - 1);
      const int NT0 = (n0 + 31) / 32, NT1 = (n1 + 31) / 32, NTs = (L + 31) / 32;
      m.nd[kind] = 1;
      m.zs[kind] = zs;
      q[0] = BandPart{NT0 + NTs, BT, NT0, 32 * NT0 - n0, n0, L, 0, 0, 0, 0, 0, 0};
      q[1] = BandPart{NT1 + NTs, BT, NT1, 32 * NT1 - n1, n1, L, 1, 0, 0, 0, 0, 0};
      q[2] = BandPart{NTs, NTs, NTs, 0, 0, L, 0, 0, 0, 0, 0, 0};
    } else {
      q[0] = BandPart{NT, BT, NT, 0, n, 0, 0, 0, 0, 0, 0, 0};
    }
  }
}

// Factor storage of every box part, the factorisation descriptors, and the
// ops and work layouts (rerun when MSGFEM_OPT_SPLIT changes).
static int plan_layout(msgfem_plan* p, int nsd, int n_mat) {
  const int nb = (int)p->meta.size(), k = p->k;
  p->max_nt = p->max_bt = 0;
  p->max_bt_kind[0] = p->max_bt_kind[1] = 0;
  p->max_fac_tiles = 0;
  p->max_nts = 0;
  p->any_split[0] = p->any_split[1] = false;
  int64_t fac_off = 0;
  for (int b = 0; b < nb; ++b) {
    BoxMeta& m = p->meta[b];
    band_parts(m, p->split != 0);
    for (int kind = 0; kind < 2; ++kind) {
      for (int pi = 0; pi < (m.nd[kind] ? 3 : 1); ++pi) {
        BandPart& q = m.part[kind][pi];
        q.off = fac_off;
        fac_off += (int64_t)q.NT * q.BT * 1024;
        q.ioff = fac_off;
        fac_off += (int64_t)q.NT * 1024;
        q.fw = fac_off;
        fac_off += solve_copy_doubles(q.NT, q.BT);
        q.bw = fac_off;
        fac_off += solve_copy_doubles(q.NT, q.BT);
        p->max_nt = std::max(p->max_nt, q.NT);
        p->max_bt = std::max(p->max_bt, q.BT);
        p->max_bt_kind[kind] = std::max(p->max_bt_kind[kind], q.BT);
        p->max_fac_tiles = std::max(p->max_fac_tiles, (int64_t)q.NT * q.BT);
      }
      if (m.nd[kind]) {
        p->any_split[kind] = true;
        p->max_nts = std::max(p->max_nts, m.part[kind][2].NT);
      }
    }
  }
  // block solve LDS: per-wavefront partial sums, D^{-1} tile, w row, ring of BT solution rows
  if (p->max_bt > SOLVE_MAX_BT ||
      (int64_t)(8 * 32 * (KC + 1) + 32 * 33 + 32 * KC + p->max_bt * 32 * KC) * 8 > 160 * 1024)
    return fail(p, MSGFEM_ESIZE, "band of %d tiles too wide for the block solve (at most %d)", p->max_bt,
                SOLVE_MAX_BT);
  // factorisation descriptors: whole bands and chains, then separator blocks
  p->mats.clear();
  p->seps.clear();
  for (int b = 0; b < nb; ++b)
    for (int kind = 0; kind < 2; ++kind) {
      const BoxMeta& m = p->meta[b];
      for (int pi = 0; pi < (m.nd[kind] ? 2 : 1); ++pi) {
        const BandPart& q = m.part[kind][pi];
        p->mats.push_back(MatDesc{q.NT, q.BT, b, q.NTf, q.off, q.ioff});
      }
    }
  p->n_chain_mats = (int)p->mats.size();
  for (int b = 0; b < nb; ++b)
    for (int kind = 0; kind < 2; ++kind) {
      const BoxMeta& m = p->meta[b];
      if (!m.nd[kind]) continue;
      const BandPart *c0 = &m.part[kind][0], *c1 = &m.part[kind][1], *q = &m.part[kind][2];
      p->mats.push_back(MatDesc{q->NT, q->BT, b, q->NTf, q->off, q->ioff});
      p->seps.push_back(SepDesc{q->NT, c0->BT, c0->NTf, c1->NTf, c0->off, c1->off, q->off});
    }
  p->fac_total = fac_off;
  // block-solve dispatch order: longest sweep (tile rows x band tiles of the
  // longest part) first
  p->order.assign((size_t)2 * nb, 0);
  for (int kind = 0; kind < 2; ++kind) {
    std::vector<std::pair<int64_t, int>> w(nb);
    for (int b = 0; b < nb; ++b) {
      const BoxMeta& m = p->meta[b];
      int64_t c = 0;
      for (int pi = 0; pi < (m.nd[kind] ? 2 : 1); ++pi)
        c = std::max(c, (int64_t)m.part[kind][pi].NT * m.part[kind][pi].BT);
      w[b] = {-c, b};
    }
    std::stable_sort(w.begin(), w.end());
    for (int b = 0; b < nb; ++b) p->order[(size_t)kind * nb + b] = w[b].second;
  }
  const msgfem_eig_opts& o = p->opts;
  // ops layout
  int64_t off = 0;
  p->o_meta = off; off = align256(off + (int64_t)nb * sizeof(BoxMeta));
  p->o_mats = off; off = align256(off + (int64_t)p->mats.size() * sizeof(MatDesc));
  p->o_seps = off; off = align256(off + (int64_t)std::max<size_t>(p->seps.size(), 1) * sizeof(SepDesc));
  p->o_order = off; off = align256(off + (int64_t)2 * nb * 4);
  p->o_omega = off; off = align256(off + (int64_t)nsd * 6 * 4);
  p->o_ctab = off; off = align256(off + (int64_t)n_mat * 36 * 8);
  p->o_wtot = off; off = align256(off + p->n_nodes_global * 4);
  p->o_stencil = off; off = align256(off + p->nodes_total * 243 * 8);
  p->o_mu = off; off = align256(off + p->dofs_total * 8);
  p->o_cls = off; off = align256(off + p->dofs_total);
  p->o_fac = off; off = align256(off + p->fac_total * 8);
  p->o_fac32 = p->o_st32 = 0;
  if (o.precision >= 1) {
    // FP32 copies of the factors' solve data (precision 1: the preconditioner's
    // Ahat only; 2: both matrices) and of the stencil (precision 2)
    p->o_fac32 = off; off = align256(off + p->fac_total * 4);
    if (o.precision == 2) { p->o_st32 = off; off = align256(off + p->nodes_total * 243 * 4); }
  }
  p->ops_bytes = off;
  // work layout
  int m3 = 3 * k;
  int nchunk_solve = (k + KC - 1) / KC;
  // w rows of the solve plus one row that absorbs stores without a target
  // (per 8 columns; a 16-column solve takes two strides per chunk)
  p->scr_stride = (int64_t)(p->max_nt + 1) * 32 * KC;
  // separator exchange of a split solve: t_0, t_1, w of S, x_s
  p->sep_q = (int64_t)(p->max_nts + 1) * 32 * KC;
  // chunks of 8 columns, rounded up to whole chunks of 16
  nchunk_solve = 2 * ((k + 15) / 16);
  off = 0;
  // 20 LOBPCG blocks, two scratch blocks, and the four image kinds of the
  // converged block of every round but the last
  p->w_vec = off; off = align256(off + (22 + 4 * (int64_t)(p->rounds - 1)) * p->vec_total * 8);
  p->w_part = off; off = align256(off + (int64_t)nb * p->n_gchunk * 2 * m3 * m3 * 8);
  p->w_G = off; off = align256(off + (int64_t)nb * 2 * m3 * m3 * 8);
  p->w_L = off; off = align256(off + (int64_t)nb * m3 * m3 * 8);
  // Rayleigh-Ritz coefficients (3k x k), or a coarse basis's CholQR
  // coefficients (kv x kv)
  p->w_Y = off; off = align256(off + (int64_t)nb * std::max(m3 * k, p->kv * p->kv) * 8);
  p->w_Yp = off; off = align256(off + (int64_t)nb * m3 * k * 8);
  p->w_nu = off; off = align256(off + (int64_t)nb * k * 8);
  p->w_rho = off; off = align256(off + (int64_t)nb * k * 8);
  p->w_rpart = off; off = align256(off + (int64_t)nb * p->n_gchunk * 3 * 32 * 8);
  p->w_active = off; off = align256(off + (int64_t)nb * 4);
  p->w_iters = off; off = align256(off + (int64_t)nb * 4);
  p->w_nact = off; off = align256(off + 8);   // active-box count, iteration index
  p->w_reached = off; off = align256(off + (int64_t)nb * 4);
  p->w_xbuf = off; off = align256(off + (int64_t)nb * 4);
  // one w block per (box, chain, chunk)
  p->w_scr = off; off = align256(off + (int64_t)2 * nb * nchunk_solve * p->scr_stride * 8);
  p->w_sep = off;
  if (p->any_split[0] || p->any_split[1]) off = align256(off + (int64_t)nb * nchunk_solve * 4 * p->sep_q * 8);
  p->work_bytes = off;
  return MSGFEM_OK;
}

extern "C" int msgfem_plan_create(msgfem_plan** out, int device, const msgfem_mesh* mesh,
                                  const msgfem_decomp* dec, const int32_t* batch,
                                  const int32_t* n_ev, int32_t nb,
                                  const msgfem_eig_opts* opts) {
  if (!out || !mesh || !dec || !batch || !n_ev || nb <= 0) return MSGFEM_EARG;
  *out = nullptr;
  msgfem_plan* p = new msgfem_plan();
  *out = p;
  p->device = device;
  p->mesh = *mesh;
  p->nsd = dec->nsd;
  p->overlap = dec->overlap;
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || mesh->n_mat < 1)
    return fail(p, MSGFEM_EARG, "bad mesh dimensions");
  if (!mesh->node_xyz || !mesh->elem_mat || !mesh->materials || !mesh->dirichlet)
    return fail(p, MSGFEM_EARG, "null mesh array");
  if (dec->nsd < 1 || !dec->cores || !dec->ovs || dec->overlap < 1)
    return fail(p, MSGFEM_EARG, "bad decomposition (nsd >= 1, overlap >= 1 required)");
  msgfem_eig_opts o;
  o.shift = 1.0; o.tol = 1e-6; o.maxit = 200; o.block = 0; o.precision = 0; o.geneo = 0; o.seed = 1234;
  if (opts) {
    o = *opts;
    if (!(o.shift > 0)) o.shift = 1.0;
    if (!(o.tol > 0)) o.tol = 1e-6;
    if (o.maxit <= 0) o.maxit = 200;
  }
  if (o.precision < 0 || o.precision > 2) return fail(p, MSGFEM_EARG, "precision %d not supported", o.precision);
  if (o.precision == 2 && o.geneo)
    return fail(p, MSGFEM_EARG, "the FP32-operator phase is for the A-harmonic GEVP only");
  p->opts = o;
  const int N[3] = {mesh->nx, mesh->ny, mesh->nz};
  p->n_nodes_global = (int64_t)(N[0] + 1) * (N[1] + 1) * (N[2] + 1);
  p->omega.resize(6 * (size_t)dec->nsd);
  for (int j = 0; j < dec->nsd; ++j) {
    const int32_t* c = dec->cores + 6 * j;
    for (int d = 0; d < 3; ++d) {
      if (c[d] < 0 || c[3 + d] > N[d] || c[d] >= c[3 + d])
        return fail(p, MSGFEM_EARG, "core %d out of the mesh", j);
      p->omega[6 * j + d] = std::max(c[d] - dec->overlap, 0);
      p->omega[6 * j + 3 + d] = std::min(c[3 + d] + dec->overlap, N[d]);
    }
  }
  int maxnev = 0;
  for (int b = 0; b < nb; ++b) maxnev = std::max(maxnev, n_ev[b]);
  if (maxnev < 1 || maxnev > MAX_NEV) return fail(p, MSGFEM_EARG, "n_ev must be in [1, %d]", MAX_NEV);
  int k = o.block;
  if (maxnev <= 32) {
    if (k <= 0) {
      // twice n_ev, at least n_ev + 8: the block solves of 8-column chunks run
      // side by side, so wider blocks cost little per iteration and cut the
      // iteration count (uniform batch: 6.9 iterations at k = 32, 8.6 at 24)
      k = std::max(2 * maxnev, maxnev + 8);
      k = (k + 7) / 8 * 8;
    }
    k = std::min(k, 32);
    if (k < maxnev) return fail(p, MSGFEM_EARG, "block %d < n_ev %d", k, maxnev);
    p->nround = maxnev;
    p->rounds = 1;
  } else {
    // deflated rounds of ROUND_PAIRS pairs with a block of 32 (8 guard columns)
    if (k > 0 && k != 32) return fail(p, MSGFEM_EARG, "n_ev > 32 runs deflated rounds with block 32 (got %d)", k);
    k = 32;
    p->nround = ROUND_PAIRS;
    p->rounds = (maxnev + ROUND_PAIRS - 1) / ROUND_PAIRS;
  }
  if (k % 2) return fail(p, MSGFEM_EARG, "block width must be even");
  p->k = k;
  p->kv = std::max(k, (maxnev + 7) / 8 * 8);
  p->meta.resize(nb);
  int64_t node_off = 0, dof_off = 0, vec_off = 0, evec_off = 0, eval_off = 0;
  for (int b = 0; b < nb; ++b) {
    int sd = batch[b];
    if (sd < 0 || sd >= dec->nsd) return fail(p, MSGFEM_EARG, "batch[%d] = %d out of range", b, sd);
    if (n_ev[b] < 1) return fail(p, MSGFEM_EARG, "n_ev[%d] < 1", b);
    if (dec->ovs[sd] < 0) return fail(p, MSGFEM_EARG, "ovs[%d] < 0", sd);
    BoxMeta m;
    if (const char* e = box_geometry(N, dec, p->omega.data(), o.geneo != 0, sd, n_ev[b], m))
      return fail(p, MSGFEM_EARG, "subdomain %d: %s", sd, e);
    m.node_off = node_off;
    m.dof_off = dof_off;
    m.vec_off = vec_off;
    m.evec_off = evec_off;
    m.eval_off = eval_off;
    node_off += m.n_nodes;
    dof_off += m.n_dof;
    vec_off += (int64_t)m.n_dof * k;
    evec_off += (int64_t)m.n_dof * m.n_ev;
    eval_off += m.n_ev;
    p->max_nodes = std::max(p->max_nodes, m.n_nodes);
    p->max_dof = std::max(p->max_dof, m.n_dof);
    p->meta[b] = m;
  }
  p->nodes_total = node_off;
  p->dofs_total = dof_off;
  p->vec_total = vec_off;
  p->evec_total = evec_off;
  p->eval_total = eval_off;
  p->n_gchunk = (p->max_dof + GRAM_ROWS - 1) / GRAM_ROWS;
  return plan_layout(p, dec->nsd, mesh->n_mat);
}

extern "C" void msgfem_plan_destroy(msgfem_plan* p) { delete p; }

extern "C" const char* msgfem_plan_error(const msgfem_plan* p) {
  return p ? p->err.c_str() : "null plan";
}

extern "C" int msgfem_plan_sizes(const msgfem_plan* p, msgfem_sizes* s) {
  if (!p || !s) return MSGFEM_EARG;
  s->ops_bytes = p->ops_bytes;
  s->work_bytes = p->work_bytes;
  s->n_eval = p->eval_total;
  s->n_evec = p->evec_total;
  s->n_dof = p->dofs_total;
  s->block = p->k;
  s->n_box = (int32_t)p->meta.size();
  return MSGFEM_OK;
}

extern "C" int msgfem_plan_box(const msgfem_plan* p, int32_t b, msgfem_box_info* o) {
  if (!p || !o || b < 0 || b >= (int32_t)p->meta.size()) return MSGFEM_EARG;
  const BoxMeta& m = p->meta[b];
  o->sd = m.sd;
  o->mx = m.mx; o->my = m.my; o->mz = m.mz;
  for (int d = 0; d < 3; ++d) o->g0[d] = m.g0[d];
  o->n_nodes = m.n_nodes;
  o->n_dof = m.n_dof;
  o->n_ev = m.n_ev;
  // class counts from geometry (host): B2 = interior faces, B3 needs the Dirichlet flags
  int n2n = 0;
  for (int kk = 0; kk < m.mz; ++kk)
    for (int jj = 0; jj < m.my; ++jj)
      for (int ii = 0; ii < m.mx; ++ii) {
        int l[3] = {ii, jj, kk}, mm[3] = {m.mx, m.my, m.mz};
        bool b2 = false;
        for (int d = 0; d < 3; ++d)
          if ((m.iface_lo[d] && l[d] == 0) || (m.iface_hi[d] && l[d] == mm[d] - 1)) b2 = true;
        n2n += b2;
      }
  o->n2 = 3 * n2n;   // before removing Dirichlet DoFs on the interior faces
  o->n1 = m.n_dof - o->n2;
  o->n3 = -1;        // needs device data (Dirichlet flags); read the class array
  o->stencil_off = p->o_stencil + m.node_off * 243 * 8;
  o->cls_off = p->o_cls + m.dof_off;
  o->mu_off = p->o_mu + m.dof_off * 8;
  o->vec_off = m.vec_off;
  o->evec_off = m.evec_off;
  o->eval_off = m.eval_off;
  return MSGFEM_OK;
}

// exact number of stored entries of a lower band of order n and half-bandwidth b
static double band_entries(double n, double b) {
  if (b > n - 1) b = n - 1;
  return n * (b + 1) - b * (b + 1) / 2;
}

static void band_nb(const BoxMeta& m, int kind, double* n, double* b) {
  int d[3];
  for (int a = 0; a < 3; ++a)
    d[a] = kind == 0 ? m.sub_hi[a] - m.sub_lo[a] + 1 : (a == 0 ? m.mx : (a == 1 ? m.my : m.mz));
  const int ord = m.ord[kind];
  const int sx = d[ord & 3], sy = d[(ord >> 2) & 3];
  *n = kind == 0 ? m.n11 : m.nh;
  *b = 3.0 * (sx * sy + sx + 1) + 2;
}

static MeshDev mesh_dev(const msgfem_plan* p) {
  MeshDev md;
  md.nx = p->mesh.nx; md.ny = p->mesh.ny; md.nz = p->mesh.nz; md.n_mat = p->mesh.n_mat;
  md.xyz = p->mesh.node_xyz; md.elem_mat = p->mesh.elem_mat; md.materials = p->mesh.materials;
  md.dirichlet = p->mesh.dirichlet;
  return md;
}

struct OpsView {
  const BoxMeta* meta;
  MatDesc* mats;
  SepDesc* seps;
  int32_t* order;
  int32_t* omega;
  double* ctab;
  int32_t* wtot;
  double* stencil;
  double* mu1;
  uint8_t* cls;
  double* fac;
  float* fac32;      // mixed path only
  float* stencil32;  // mixed path only
};

static OpsView ops_view(const msgfem_plan* p, const void* ops) {
  char* b = (char*)ops;
  OpsView v;
  v.meta = (const BoxMeta*)(b + p->o_meta);
  v.mats = (MatDesc*)(b + p->o_mats);
  v.seps = (SepDesc*)(b + p->o_seps);
  v.order = (int32_t*)(b + p->o_order);
  v.omega = (int32_t*)(b + p->o_omega);
  v.ctab = (double*)(b + p->o_ctab);
  v.wtot = (int32_t*)(b + p->o_wtot);
  v.stencil = (double*)(b + p->o_stencil);
  v.mu1 = (double*)(b + p->o_mu);
  v.cls = (uint8_t*)(b + p->o_cls);
  v.fac = (double*)(b + p->o_fac);
  v.fac32 = p->o_fac32 ? (float*)(b + p->o_fac32) : nullptr;
  v.stencil32 = p->o_st32 ? (float*)(b + p->o_st32) : nullptr;
  return v;
}

static void lds_attributes();

// the matrix-core block solve serves a matrix kind whose bands all fit its slots
// block-solve family of a matrix kind (MSGFEM_OPT_SOLVE: 0 widest that fits,
// 1 vector FMA, 2 matrix cores with 8 columns, 3 matrix cores with 16 columns)
static bool solve4_kind(const msgfem_plan* p, int kind) {
  return p->solve_pref != 1 && p->max_bt_kind[kind] - 1 <= 8 * SOLVE4_MAX_SLOTS;
}

// the wide (16-column) matrix-core solve for this matrix kind
static bool wide_kind(const msgfem_plan* p, int kind) {
  return solve4_kind(p, kind) && p->solve_pref != 2 && p->max_bt_kind[kind] <= WIDE_MAX_BT;
}

static int set_device(msgfem_plan* p) {
  HIPCHK(p, hipSetDevice(p->device));
  lds_attributes();
  return MSGFEM_OK;
}

// Tile Cholesky of a list of SPD matrices in tile-band storage: per tile column
// one update launch (which also factors the next diagonal tile) and one panel
// launch, then the block unit-lower rewrite A = Lu D Lu^T.
static int tile_cholesky(msgfem_plan* p, const MatDesc* mats, int nmat, int max_nt, int max_bt,
                         double* fac, int32_t* status, hipStream_t s) {
  const int mmax = max_bt - 1;
  const int upd_wg = std::max(1, (mmax * (mmax + 1) / 2 + 3) / 4);
  const int pan_wg = std::max(1, (mmax + 3) / 4);
  for (int K = -1; K < max_nt - 1; ++K) {
    k_chol_update<<<dim3(K < 0 ? 1 : upd_wg, nmat), 256, 0, s>>>(mats, K, fac, status);
    k_chol_panel<<<dim3(pan_wg, nmat), 256, 0, s>>>(mats, K + 1, fac);
  }
  k_chol_unit<<<dim3((unsigned)(((int64_t)max_nt * max_bt + 3) / 4), nmat), 256, 0, s>>>(mats, fac);
  LAUNCHCHK(p);
  return 0;
}

// Single-RHS solve with the dense unit-lower tile factor (BT = NT): x = A^{-1} b
// (b of length NH, y and x of NT*32 doubles) by column launches over many
// workgroups (k_trsv_*).
static int tile_trsv(const double* T, int NT, int NH, const double* b, double* y, double* x, hipStream_t s) {
  k_trsv_init<<<(NT * 32 + 255) / 256, 256, 0, s>>>(b, NH, NT * 32, y);
  for (int J = 0; J < NT - 1; ++J) k_trsv_fwd<<<NT - 1 - J, 256, 0, s>>>(T, NT, J, y);
  k_trsv_diag<<<NT, 256, 0, s>>>(T, NT, y, x);
  for (int J = NT - 1; J >= 1; --J) k_trsv_bwd<<<J, 256, 0, s>>>(T, NT, J, x);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

// Left-looking tile Cholesky of banded SPD matrices, one launch per tile
// column (which also factors the next diagonal tile), then (unit) the block
// unit-lower rewrite.
// steps J = -1 .. last_J of k_chol_step (last_J = NT - 2 for a whole band,
// NTf - 1 for a chain, whose last step gives its separator rows' L tiles)
static int band_cholesky(msgfem_plan* p, const MatDesc* mats, int nmat, int last_J, int max_nt, int max_bt,
                         double* fac, int32_t* status, bool unit, hipStream_t s) {
  // one workgroup per matrix for all steps (MSGFEM_OPT_CHOL 2, or by default
  // when the matrices fill the CUs about once and the bands are narrow, so
  // that a step's jobs suit 8 wavefronts: uniform batch, 256 matrices of
  // 24-tile bands, 35.0 -> 33.7 ms per factor pass), else a launch per step
  bool per_matrix = p->chol_pref == 2;
  if (p->chol_pref == 0) {
    if (p->n_cu == 0 && hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
      p->n_cu = -1;
    per_matrix = p->n_cu > 0 && nmat <= p->n_cu && 4 * nmat >= 3 * p->n_cu && max_bt <= 24;
  }
  if (per_matrix) {
    k_chol_matrix<CHOL_PANEL><<<nmat, 512, 0, s>>>(mats, last_J, fac, status);
  } else {
    // row workgroups in groups of 8 matrices for bands wider than 24 tiles
    // (a matrix's rows then share its tiles in L2: uneven batch, 41-tile
    // bands, 146 -> 140 ms per factor pass), else the longest rows of every
    // matrix first (uniform batch, 24-tile bands: groups of 8 take 36.5 ms,
    // not 35.0)
    const int group = max_bt > 24 ? 8 : (nmat + 7) / 8 * 8;
    for (int J = -1; J <= last_J; ++J)
      k_chol_step<CHOL_PANEL><<<chol_grid(CHOL_PANEL, nmat, max_bt), 256, 0, s>>>(mats, nmat, max_bt, group, J, fac,
                                                                                    status);
  }
  if (unit) k_chol_unit<<<dim3((unsigned)(((int64_t)max_nt * max_bt + 3) / 4), nmat), 256, 0, s>>>(mats, fac);
  LAUNCHCHK(p);
  return 0;
}

extern "C" int msgfem_assemble_local(msgfem_plan* p, void* ops, int32_t* status, void* stream) {
  if (!p || !ops || !status) return fail(p, MSGFEM_EARG, "null argument");
  if (set_device(p)) return MSGFEM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  OpsView v = ops_view(p, ops);
  const int nb = (int)p->meta.size();
  HIPCHK(p, hipMemcpyAsync((void*)v.meta, p->meta.data(), nb * sizeof(BoxMeta), hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(v.omega, p->omega.data(), p->omega.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(v.mats, p->mats.data(), p->mats.size() * sizeof(MatDesc),
                           hipMemcpyHostToDevice, s));
  if (!p->seps.empty())
    HIPCHK(p, hipMemcpyAsync(v.seps, p->seps.data(), p->seps.size() * sizeof(SepDesc), hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(v.order, p->order.data(), p->order.size() * 4, hipMemcpyHostToDevice, s));
  // the host copies must stay alive until the copies complete
  HIPCHK(p, hipStreamSynchronize(s));
  k_fill_i32<<<(nb + 255) / 256, 256, 0, s>>>(status, nb, 0);
  LAUNCHCHK(p);
  k_materials<<<(p->mesh.n_mat + 63) / 64, 64, 0, s>>>(p->mesh.materials, p->mesh.n_mat, v.ctab);
  LAUNCHCHK(p);
  k_fill_i32<<<1024, 256, 0, s>>>(v.wtot, p->n_nodes_global, 0);
  LAUNCHCHK(p);
  int maxo = 1;
  for (int j = 0; j < p->nsd; ++j) {
    const int32_t* o = &p->omega[6 * j];
    maxo = std::max(maxo, (o[3] - o[0] + 1) * (o[4] - o[1] + 1) * (o[5] - o[2] + 1));
  }
  {
    dim3 grid((maxo + 255) / 256, p->nsd);
    k_pou_total<<<grid, 256, 0, s>>>(v.omega, p->nsd, p->mesh.nx, p->mesh.ny, p->mesh.nz,
                                     2 * p->overlap, v.wtot);
    LAUNCHCHK(p);
  }
  MeshDev md = mesh_dev(p);
  {
    dim3 grid((p->max_nodes + 3) / 4, nb);
    double by = 0;
    for (auto& m : p->meta) by += 243.0 * 8 * m.n_nodes;
    ProfScope ps(p, PK_ASSEMBLE, s, by, 0.0);
    k_assemble<<<grid, 256, 0, s>>>(v.meta, md, v.ctab, v.stencil);
    LAUNCHCHK(p);
  }
  {
    dim3 grid((p->max_nodes + 255) / 256, nb);
    k_classes_mu<<<grid, 256, 0, s>>>(v.meta, md, 2 * p->overlap, v.wtot, v.cls, v.mu1);
    LAUNCHCHK(p);
  }
  // batches whose bands all fit the matrix-core solve take the unit-lower
  // rewrite inside the copies (k_band_unit_relayout4)
  const bool fused_unit = solve4_kind(p, 0) && solve4_kind(p, 1);
  for (int kind = 0; kind < 2; ++kind) {
    int64_t tot = p->max_fac_tiles * 128;
    int64_t blocks = std::min<int64_t>((tot + 255) / 256, 65535);
    dim3 grid((unsigned)blocks, nb, p->any_split[kind] ? 3 : 1);
    double by = 0;
    for (auto& m : p->meta) {
      double n, b;
      band_nb(m, kind, &n, &b);
      by += 8.0 * band_entries(n, b);
    }
    ProfScope ps(p, PK_BUILD, s, by, 0.0);
    k_band_build<<<grid, 256, 0, s>>>(v.meta, kind, v.stencil, v.cls, v.mu1, p->opts.shift, v.fac);
    LAUNCHCHK(p);
  }
  {
    double by = 0, fl = 0;
    for (auto& m : p->meta) {
      for (int kind = 0; kind < 2; ++kind) {
        double n, b;
        band_nb(m, kind, &n, &b);
        by += 2 * 8.0 * band_entries(n, b);
        fl += n * b * b - 2.0 / 3.0 * b * b * b;
      }
    }
    ProfScope ps(p, PK_POTRF, s, by, fl);
    // whole bands and chains (a chain stops at its separator rows), the
    // separators' Schur complements, then the separator blocks
    int last_J = -1, max_nt = 0, max_bt = 0;
    for (int i = 0; i < p->n_chain_mats; ++i) {
      const MatDesc& d = p->mats[i];
      last_J = std::max(last_J, d.NTf < d.NT ? d.NTf - 1 : d.NT - 2);
      max_nt = std::max(max_nt, d.NT);
      max_bt = std::max(max_bt, d.BT);
    }
    const int nsep = (int)p->seps.size();
    // the separators' Schur complements read the chains' Cholesky tiles, so
    // the unit-lower rewrite of the chains (when not fused into the copies)
    // comes after them
    if (band_cholesky(p, v.mats, p->n_chain_mats, last_J, max_nt, max_bt, v.fac, status, !fused_unit && !nsep, s))
      return MSGFEM_EHIP;
    if (nsep) {
      const int nts = p->max_nts;
      const int ntg = (nts * (nts + 1) / 2 + 3) / 4;
      k_sep_syrk<<<8 * ntg * ((nsep + 7) / 8), 256, 0, s>>>(v.seps, nsep, ntg, v.fac);
      LAUNCHCHK(p);
      if (!fused_unit) {
        k_chol_unit<<<dim3((unsigned)(((int64_t)max_nt * max_bt + 3) / 4), p->n_chain_mats), 256, 0, s>>>(v.mats,
                                                                                                         v.fac);
        LAUNCHCHK(p);
      }
      if (band_cholesky(p, v.mats + p->n_chain_mats, nsep, nts - 2, nts, nts, v.fac, status, !fused_unit, s))
        return MSGFEM_EHIP;
    }
  }
  for (int kind = 0; kind < 2; ++kind) {
    int max_nt = 1, max_sets = 1;
    double by = 0;
    for (auto& m : p->meta)
      for (int pi = 0; pi < (m.nd[kind] ? 3 : 1); ++pi) {
        const BandPart& q = m.part[kind][pi];
        max_nt = std::max(max_nt, q.NT);
        max_sets = std::max(max_sets, solve_sets(q.BT));
        by += 3 * 8.0 * solve_copy_doubles(q.NT, q.BT);
      }
    ProfScope ps(p, PK_BUILD, s, by, 0.0);
    const unsigned nz = (unsigned)(3 * nb);
    const int wide = wide_kind(p, kind) ? 1 : 0;
    if (fused_unit)
      k_band_unit_relayout4<<<dim3((solve4_slots(p->max_bt_kind[kind]) + 3) / 4, max_nt, nz), 256, 0, s>>>(
          v.meta, kind, v.fac, wide);
    else if (solve4_kind(p, kind))
      k_band_relayout4<<<dim3(solve4_slots(p->max_bt_kind[kind]), max_nt, nz), 256, 0, s>>>(v.meta, kind, v.fac,
                                                                                             wide);
    else
      k_band_relayout<<<dim3(SOLVE_TILES * max_sets, max_nt, nz), 256, 0, s>>>(v.meta, kind, v.fac);
    LAUNCHCHK(p);
  }
  if (p->opts.precision >= 1) {
    ProfScope ps(p, PK_BUILD, s, 0.0, 0.0);
    if (p->opts.precision == 1)
      k_mixed_copies<<<dim3(1024, nb, 1), 256, 0, s>>>(v.meta, 1, v.fac, v.fac32, v.stencil, v.stencil32);
    else
      k_mixed_copies<<<dim3(1024, nb, 3), 256, 0, s>>>(v.meta, 0, v.fac, v.fac32, v.stencil, v.stencil32);
    LAUNCHCHK(p);
  }
  return MSGFEM_OK;
}

// ---------------------------------------------------------------------------
// LOBPCG driver

namespace {
struct Work {
  double* vec;       // 22 block arrays of vec_total doubles
  double* part;
  double* G;
  double* L;
  double* Y;
  double* Yp;
  double* nu;
  double* rho;
  double* rpart;
  int32_t* active;
  int32_t* iters;
  int32_t* nact;
  int32_t* reached;
  int32_t* xbuf;
  double* scr;
  double* sep;
};
}  // namespace

static Work work_view(const msgfem_plan* p, void* work) {
  char* b = (char*)work;
  Work w;
  w.vec = (double*)(b + p->w_vec);
  w.part = (double*)(b + p->w_part);
  w.G = (double*)(b + p->w_G);
  w.L = (double*)(b + p->w_L);
  w.Y = (double*)(b + p->w_Y);
  w.Yp = (double*)(b + p->w_Yp);
  w.nu = (double*)(b + p->w_nu);
  w.rho = (double*)(b + p->w_rho);
  w.rpart = (double*)(b + p->w_rpart);
  w.active = (int32_t*)(b + p->w_active);
  w.iters = (int32_t*)(b + p->w_iters);
  w.nact = (int32_t*)(b + p->w_nact);
  w.reached = (int32_t*)(b + p->w_reached);
  w.xbuf = (int32_t*)(b + p->w_xbuf);
  w.scr = (double*)(b + p->w_scr);
  w.sep = (double*)(b + p->w_sep);
  return w;
}

struct Ctx {
  msgfem_plan* p;
  OpsView v;
  Work w;
  hipStream_t s;
  int nb, k;
  bool use32 = false;           // FP32 operator copies (precision 2, first phase)
  bool pre32 = false;           // FP32 copy of Ahat for the preconditioner solve (precision 1)
  bool no_alloc = false;        // the static-scratch entry point: no event objects for profiling
  std::vector<int32_t> act_h;   // host copy of the active flags (all 1 when unknown)
  bool counts(int b, const int32_t* act) const { return !act || act_h.empty() || act_h[b]; }
};

// Kernels whose dynamic LDS may exceed 64 KiB declare it once per process
// (plans may be driven from several host threads: the first caller sets the
// attributes, the others wait until it has).
static void lds_attributes_once();
static void lds_attributes() {
  static std::once_flag once;
  std::call_once(once, lds_attributes_once);
}
static void lds_attributes_once() {
  (void)hipFuncSetAttribute((const void*)k_rayleigh_ritz, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  const void* solves[4] = {(const void*)k_band_solve<KC, 1, double>, (const void*)k_band_solve<KC, 2, double>,
                           (const void*)k_band_solve<KC, 1, float>, (const void*)k_band_solve<KC, 2, float>};
  for (const void* f : solves) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  const void* solves4[16] = {
      (const void*)k_band_solve4<1, false, double>, (const void*)k_band_solve4<2, false, double>,
      (const void*)k_band_solve4<3, false, double>, (const void*)k_band_solve4<4, false, double>,
      (const void*)k_band_solve4<1, false, float>,  (const void*)k_band_solve4<2, false, float>,
      (const void*)k_band_solve4<3, false, float>,  (const void*)k_band_solve4<4, false, float>,
      (const void*)k_band_solve4<1, true, double>,  (const void*)k_band_solve4<2, true, double>,
      (const void*)k_band_solve4<3, true, double>,  (const void*)k_band_solve4<4, true, double>,
      (const void*)k_band_solve4<1, true, float>,   (const void*)k_band_solve4<2, true, float>,
      (const void*)k_band_solve4<3, true, float>,   (const void*)k_band_solve4<4, true, float>};
  for (const void* f : solves4) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_band_solve4<5, false, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_band_solve4<5, false, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_band_solve4<8, false, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_band_solve4<8, false, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_update<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  const void* spp[] = {(const void*)k_spmm_planes<false, double>, (const void*)k_spmm_planes<true, double>,
                       (const void*)k_spmm_planes<false, float>, (const void*)k_spmm_planes<true, float>};
  for (const void* f : spp) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)hipFuncSetAttribute((const void*)k_update<6>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipGetLastError();
}

static int spmm(Ctx& c, const double* X, double* Y, double* Y2, int kk, int yclasses, double scale,
                const int32_t* active) {
  const int cw = Y2 ? 4 : (kk == 1 ? 1 : 8);
  const int nq = (kk + cw - 1) / cw;
  const int bpb = (int)(((int64_t)c.p->max_nodes * nq + 255) / 256);
  dim3 grid((unsigned)(c.nb == 1 ? bpb : 8 * ((c.nb + 7) / 8) * bpb));
  double by = 0, fl = 0;
  for (int b = 0; b < c.nb; ++b) {
    if (!c.counts(b, active)) continue;
    const BoxMeta& m = c.p->meta[b];
    int nout = (Y ? 1 : 0) + (Y2 ? 1 : 0);
    by += 243.0 * 8 * m.n_nodes + 8.0 * m.n_dof * kk * (1 + nout);
    fl += 2.0 * 243 * m.n_nodes * kk * (Y2 ? 2 : 1);
  }
  ProfScope ps(c.p, PK_SPMM, c.s, by, fl, !c.no_alloc);
  // blocks of whole 8-column groups: the LDS-staged plane sweep, by default
  // (MSGFEM_OPT_SPMM 0) when the batch gives every CU a workgroup (boxes x
  // column groups >= 256) and each node plane fits one LDS tile, on request
  // (2) wherever it applies, with x-tiles for wider planes
  int max_tiles = 0;
  const int pref = c.p->spmm_pref;
  if (kk % 8 == 0 && pref != 1 && (pref == 2 || (int64_t)c.nb * (kk / 8) >= 256)) {
    for (int b = 0; b < c.nb; ++b) {
      const BoxMeta& m = c.p->meta[b];
      const int tx = sp_tile_x_host(m.mx, m.my);
      if (tx == 0) {
        max_tiles = 0;
        break;
      }
      max_tiles = std::max(max_tiles, (m.mx + tx - 1) / tx);
    }
    if (pref == 0 && max_tiles > 1) max_tiles = 0;
  }
  if (max_tiles > 0) {
    const int ng = kk / 8;
    const int64_t units = (int64_t)c.nb * max_tiles;
    const dim3 pg((unsigned)(8 * ng * ((units + 7) / 8)));
    auto launch_p = [&](auto st) {
      if (Y2)
        k_spmm_planes<true><<<pg, 1024, sp_lds(true), c.s>>>(c.v.meta, c.nb, max_tiles, ng, st, c.v.cls, c.v.mu1,
                                                            X, Y, Y2, kk, yclasses, scale, active);
      else
        k_spmm_planes<false><<<pg, 1024, sp_lds(false), c.s>>>(c.v.meta, c.nb, max_tiles, ng, st, c.v.cls,
                                                              c.v.mu1, X, Y, Y2, kk, yclasses, scale, active);
    };
    if (c.use32) launch_p((const float*)c.v.stencil32);
    else launch_p((const double*)c.v.stencil);
    LAUNCHCHK(c.p);
    return 0;
  }
  auto launch = [&](auto st) {
    if (Y2)
      k_spmm<true, 4><<<grid, 256, 0, c.s>>>(c.v.meta, c.nb, bpb, st, c.v.cls, c.v.mu1, X, Y, Y2, kk, yclasses,
                                             scale, active);
    else if (kk == 1)
      k_spmm<false, 1><<<grid, 256, 0, c.s>>>(c.v.meta, c.nb, bpb, st, c.v.cls, c.v.mu1, X, Y, Y2, kk, yclasses,
                                              scale, active);
    else
      k_spmm<false, 8><<<grid, 256, 0, c.s>>>(c.v.meta, c.nb, bpb, st, c.v.cls, c.v.mu1, X, Y, Y2, kk, yclasses,
                                              scale, active);
  };
  if (c.use32) launch((const float*)c.v.stencil32);
  else launch((const double*)c.v.stencil);
  LAUNCHCHK(c.p);
  return 0;
}

static int solve(Ctx& c, int kind, const double* in, double* out, int kk, int out_classes, int zero_rest,
                 const int32_t* active) {
  // the preconditioner's matrix (kind 1) from its FP32 copy under precision 1
  const bool f32 = c.use32 || (kind == 1 && c.pre32);
  const bool wide = wide_kind(c.p, kind);
  const int kc = wide ? 16 : KC;
  const int nchunk = (kk + kc - 1) / kc;
  const size_t lds = (size_t)c.p->max_bt_kind[kind] * 32 * kc * 8;
  // a 16-column chunk takes the scratch of two 8-column chunks
  const int64_t scr_stride = c.p->scr_stride * (kc / KC), sep_q = c.p->sep_q * (kc / KC);
  double by = 0, fl = 0;
  for (int b = 0; b < c.nb; ++b) {
    if (!c.counts(b, active)) continue;
    double n, bw;
    band_nb(c.p->meta[b], kind, &n, &bw);
    double e = band_entries(n, bw);
    by += 2 * 8.0 * e + 2 * 8.0 * n * kk;
    fl += 4.0 * e * kk;
  }
  ProfScope ps(c.p, PK_SOLVE, c.s, by, fl, !c.no_alloc);
  // bands wider than SOLVE_TILES + 1 tiles take two tile sets per step
  const bool two = c.p->max_bt_kind[kind] - 1 > SOLVE_TILES;
  // one launch (phase 0) without split boxes, else chains forward (two units
  // per box), separator blocks, chains backward
  const bool split = c.p->any_split[kind];
  auto launch = [&](auto kern, auto ft) {
    for (int ph = split ? 1 : 0; ph <= (split ? 3 : 0); ++ph) {
      const int nun = (ph == 1 || ph == 3) ? 2 * c.nb : c.nb;
      dim3 grid(8 * nchunk * ((nun + 7) / 8));
      kern<<<grid, 512, lds, c.s>>>(c.v.meta, c.nb, nchunk, kind, ft, c.v.cls, in, out, kk, out_classes, zero_rest,
                                    c.w.scr, scr_stride, active, ph, c.w.sep, sep_q,
                                    c.v.order + (size_t)kind * c.nb);
    }
  };
  if (solve4_kind(c.p, kind)) {
    // bands of at most 65 tiles: the matrix-core solve, 1..5 tile slots per
    // wavefront, 6..8 as two sets of four (8 columns only beyond 4 slots:
    // the 16-column solve takes <= 31 tiles)
    const int ns = solve4_nslot(c.p->max_bt_kind[kind]);
    auto pick = [&](auto wide_tag, auto ft) {
      constexpr bool W = decltype(wide_tag)::value;
      typedef typename std::remove_const<typename std::remove_pointer<decltype(ft)>::type>::type FT;
      if (ns <= 1) launch(k_band_solve4<1, W, FT>, ft);
      else if (ns == 2) launch(k_band_solve4<2, W, FT>, ft);
      else if (ns == 3) launch(k_band_solve4<3, W, FT>, ft);
      else if (ns == 4 || W) launch(k_band_solve4<4, W, FT>, ft);
      else if constexpr (!W) {
        if (ns == 5) launch(k_band_solve4<5, false, FT>, ft);
        else launch(k_band_solve4<8, false, FT>, ft);
      }
    };
    if (f32) {
      const float* f = (const float*)c.v.fac32;
      if (wide) pick(std::true_type(), f);
      else pick(std::false_type(), f);
    } else {
      const double* f = (const double*)c.v.fac;
      if (wide) pick(std::true_type(), f);
      else pick(std::false_type(), f);
    }
  } else if (f32) {
    if (two) launch(k_band_solve<KC, 2, float>, (const float*)c.v.fac32);
    else launch(k_band_solve<KC, 1, float>, (const float*)c.v.fac32);
  } else {
    if (two) launch(k_band_solve<KC, 2, double>, (const double*)c.v.fac);
    else launch(k_band_solve<KC, 1, double>, (const double*)c.v.fac);
  }
  LAUNCHCHK(c.p);
  return 0;
}

// Z~ <- [E Z; Z] for a boundary block Z (B1 part written), AZ, BZ, MZ
static int harmonic_images(Ctx& c, double* Z, double* AZ, double* BZ, double* MZ, double* tmp,
                           const int32_t* act) {
  const int k = c.k;
  // extension: A11 u = -(A Z)_1
  if (spmm(c, Z, tmp, nullptr, k, 1 << 1, -1.0, act)) return MSGFEM_EHIP;
  if (solve(c, 0, tmp, Z, k, 1 << 1, 0, act)) return MSGFEM_EHIP;
  // A Z~ (B1 u B2) and D A D Z~
  if (spmm(c, Z, AZ, BZ, k, (1 << 1) | (1 << 2), 1.0, act)) return MSGFEM_EHIP;
  // adjoint: M Z = E^T (DAD Z~)_1 = -A21 A11^{-1} (DAD Z~)_1
  if (solve(c, 0, BZ, tmp, k, 1 << 1, 1, act)) return MSGFEM_EHIP;
  if (spmm(c, tmp, MZ, nullptr, k, 1 << 2, -1.0, act)) return MSGFEM_EHIP;
  return 0;
}

// Gram matrices G_S = Z~^T A Z~ and G_M = Z~^T (D A D) Z~ of the blocks
// [Z_0 .. Z_{nblk-1}] into c.w.G ([box][2][m][m], m = nblk k)
static int gram_only(Ctx& c, int nblk, double* const* Zb, double* const* AZb, double* const* BZb,
                     const int32_t* act) {
  const int k = c.k, m = nblk * k;
  Blk3 Z, A, B;
  for (int i = 0; i < 3; ++i) {
    Z.p[i] = i < nblk ? Zb[i] : nullptr;
    A.p[i] = i < nblk ? AZb[i] : nullptr;
    B.p[i] = i < nblk ? BZb[i] : nullptr;
  }
  double by = 0, fl = 0;
  for (int b = 0; b < c.nb; ++b) {
    if (!c.counts(b, act)) continue;
    const BoxMeta& mt = c.p->meta[b];
    by += 3 * 8.0 * mt.n_dof * m;
    fl += 2 * 2.0 * mt.n_dof * m * m;
  }
  ProfScope ps(c.p, PK_GRAM, c.s, by, fl);
  gram_partials(m, c.p->n_gchunk, c.nb, c.s, c.v.meta, nblk, Z, A, B, k, c.w.part, act);
  LAUNCHCHK(c.p);
  dim3 g2((2 * m * m + 255) / 256, c.nb);
  k_gram_reduce<<<g2, 256, 0, c.s>>>(m, c.p->n_gchunk, c.w.part, c.w.G, act);
  LAUNCHCHK(c.p);
  return 0;
}

static int gram(Ctx& c, int nblk, double* const* Zb, double* const* AZb, double* const* BZb,
                const int32_t* act) {
  const int k = c.k, m = nblk * k;
  if (gram_only(c, nblk, Zb, AZb, BZb, act)) return MSGFEM_EHIP;
  size_t lds_rr = ((size_t)2 * m * (m + 1) + 4 * m + 256) * 8 + ((size_t)5 * m + 1) * 4;
  // per box: the two m x m Gram matrices in, the k-column coefficient blocks
  // of X and P and k Ritz values out; flops a nominal 50 m^3 (the Cholesky
  // reduction C = L^{-1} G_M L^{-T}, about 4 m^3, and some six two-sided
  // Jacobi sweeps of about 7 m^3 each)
  double by_rr = 0.0, fl_rr = 0.0;
  for (int b = 0; b < c.nb; ++b) {
    if (!c.counts(b, act)) continue;
    by_rr += 8.0 * (2.0 * m * m + 2.0 * m * k + k);
    fl_rr += 50.0 * m * (double)m * m;
  }
  ProfScope ps2(c.p, PK_RR, c.s, by_rr, fl_rr);
  k_rayleigh_ritz<<<c.nb, 1024, lds_rr, c.s>>>(m, k, 1, c.p->opts.shift, c.w.G, c.w.L, c.w.Y, c.w.Yp,
                                               c.w.nu, act);
  LAUNCHCHK(c.p);
  return 0;
}

static uint64_t round_seed(uint64_t seed, int r) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(r + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int local_eigs_impl(msgfem_plan* p, const void* ops, void* work, const double* x0, const int32_t* mask,
                           double* evals, double* evecs, double* resid, int32_t* iters, int32_t* status,
                           void* stream) {
  if (!p || !ops || !work || !evals || !evecs || !resid || !iters || !status)
    return fail(p, MSGFEM_EARG, "null argument");
  if (set_device(p)) return MSGFEM_EHIP;
  Ctx c;
  c.p = p;
  c.v = ops_view(p, ops);
  c.w = work_view(p, work);
  c.s = (hipStream_t)stream;
  c.nb = (int)p->meta.size();
  c.k = p->k;
  const int k = c.k, nb = c.nb;
  const int64_t VT = p->vec_total;
  // block arrays: kind (0 Z~, 1 AZ~, 2 DAD Z~, 3 MZ) x slot (0 X, 1 W, 2 P, 3 Xn, 4 Pn)
  double* B[4][5];
  for (int kind = 0; kind < 4; ++kind)
    for (int sl = 0; sl < 5; ++sl) B[kind][sl] = c.w.vec + (int64_t)(kind * 5 + sl) * VT;
  double* tmp = c.w.vec + (int64_t)20 * VT;
  // converged blocks of the earlier rounds, four image kinds each
  auto Yblk = [&](int r, int kind) { return c.w.vec + (int64_t)(22 + 4 * r + kind) * VT; };
  int32_t* act = c.w.active;
  // A-harmonic GEVP: unknowns on B2, images through the extension; GenEO: all
  // of B1 u B2, M = D A D itself (kind 2 doubles as M Z)
  const bool geneo = p->opts.geneo != 0;
  const int vcls = geneo ? ((1 << 1) | (1 << 2)) : (1 << 2);
  const int nkinds = geneo ? 3 : 4;
  const dim3 ugrid((unsigned)((p->max_dof + UPD_ROWS - 1) / UPD_ROWS), nb, nkinds);
  auto images = [&](double* Z, double* AZ, double* BZ, double* MZ, const int32_t* a_) -> int {
    if (geneo) return spmm(c, Z, AZ, BZ, k, (1 << 1) | (1 << 2), 1.0, a_);
    return harmonic_images(c, Z, AZ, BZ, MZ, tmp, a_);
  };
  k_fill_i32<<<(nb + 255) / 256, 256, 0, c.s>>>(c.w.iters, nb, 0);
  // bits of an earlier solve of the same boxes are stale (bit 4 of the assembly stays)
  k_status_clear<<<(nb + 255) / 256, 256, 0, c.s>>>(nb, mask, status);
  LAUNCHCHK(p);
  // a caller mask solves only the boxes it selects; the others are inactive
  // from the start and their outputs are left as they are
  std::vector<int32_t> mask_h(nb, 1);
  if (mask) {
    HIPCHK(p, hipMemcpyAsync(mask_h.data(), mask, nb * 4, hipMemcpyDeviceToHost, c.s));
    HIPCHK(p, hipStreamSynchronize(c.s));
    for (int b = 0; b < nb; ++b) mask_h[b] = mask_h[b] != 0;
  }
  // Rayleigh-Ritz on X alone (T-orthonormalises the block; also used when the
  // mixed path moves to the FP64 operators)
  auto rr_x = [&](const int32_t* a_) -> int {
    double* Zb[1] = {B[0][0]};
    double* Ab[1] = {B[1][0]};
    double* Bb[1] = {B[2][0]};
    if (gram(c, 1, Zb, Ab, Bb, a_)) return MSGFEM_EHIP;
    Blk4x3 Z;
    Out4 OX, OP;
    for (int kind = 0; kind < 4; ++kind) {
      Z.p[kind][0] = B[kind][0];
      Z.p[kind][1] = Z.p[kind][2] = nullptr;
      OX.p[kind] = B[kind][3];
      OP.p[kind] = nullptr;
    }
    k_update<2><<<ugrid, UPD_THREADS, upd_lds(k, 2), c.s>>>(c.v.meta, 1, k, Z, OX, OP, c.w.Y, c.w.Yp, a_);
    LAUNCHCHK(p);
    for (int kind = 0; kind < 4; ++kind) std::swap(B[kind][0], B[kind][3]);
    return 0;
  };
  // Deflation: block slot sl (all image kinds) made T-orthogonal to the
  // converged blocks of rounds 0 .. r-1 (classical Gram-Schmidt against each,
  // through the T-Gram cross block), the result swapped into slot sl
  auto deflate = [&](int r, int sl, const int32_t* a_) -> int {
    for (int q = 0; q < r; ++q) {
      double* Zb[2] = {B[0][sl], Yblk(q, 0)};
      double* Ab[2] = {B[1][sl], Yblk(q, 1)};
      double* Bb[2] = {B[2][sl], Yblk(q, 2)};
      if (gram_only(c, 2, Zb, Ab, Bb, a_)) return MSGFEM_EHIP;
      k_proj_coef<<<nb, 256, 0, c.s>>>(k, p->opts.shift, c.w.G, c.w.Y, a_);
      Blk4x3 Z;
      Out4 OX, OP;
      for (int kind = 0; kind < 4; ++kind) {
        Z.p[kind][0] = B[kind][sl];
        Z.p[kind][1] = Yblk(q, kind);
        Z.p[kind][2] = nullptr;
        OX.p[kind] = B[kind][3];
        OP.p[kind] = nullptr;
      }
      k_update<2><<<ugrid, UPD_THREADS, upd_lds(2 * k, 2), c.s>>>(c.v.meta, 2, k, Z, OX, OP, c.w.Y, c.w.Yp,
                                                                         a_);
      LAUNCHCHK(p);
      for (int kind = 0; kind < 4; ++kind) std::swap(B[kind][sl], B[kind][3]);
    }
    return 0;
  };
  const int n_chunk = p->n_gchunk;
  const int nround = p->nround;
  // target of the rounds that later rounds deflate against (see k_converge)
  // (not below 1e-10: the FP64 images' rounding floor, below which an
  // unlocked column's preconditioned residual is noise)
  const double tol_defl = std::max(1e-4 * p->opts.tol, 1e-10);
  // Precision 2: the first phase runs the SpMM and the block solves with FP32
  // operator copies (FP64 arithmetic and FP64 dense steps); once every active
  // box has rho <= switch_tol (or the FP32 phase stagnates, or after fp32_cap
  // iterations) the block X is re-imaged with the FP64 operators,
  // re-orthonormalised, and the iteration continues in FP64 (without the P
  // block once) to the requested tolerance, so the final residual check is
  // FP64.  Precision 1: the preconditioner solve reads its FP32 copy.
  const bool mixed = p->opts.precision == 2;
  c.pre32 = p->opts.precision == 1;
  const double switch_tol = std::max(1e-4, 100.0 * p->opts.tol);
  const int fp32_cap = 30;
  std::vector<double> rho_h, rhist;
  // Round r finds the pairs r*nround .. r*nround + nround - 1 of every box that
  // has that many (one round when n_ev <= 32), its block kept T-orthogonal to
  // the converged blocks of the earlier rounds
  int32_t* it_dev = c.w.nact + 1;   // the iteration index k_converge sees
  // physical buffer id (0..4) of a slot (the same for every image kind)
  auto buf_id = [&](int sl) { return (int)((B[0][sl] - c.w.vec) / VT); };
  const bool use_graph = p->graph_mode != 0 && !p->prof_on;
  p->graph_launches = p->graph_iters = 0;
  for (int r = 0; r < p->rounds; ++r) {
    const int col0 = r * nround;
    std::vector<int32_t> act_r(nb);
    int n_r = 0;
    for (int b = 0; b < nb; ++b) {
      act_r[b] = mask_h[b] && p->meta[b].n_ev > col0;
      n_r += act_r[b];
    }
    if (n_r == 0) break;
    HIPCHK(p, hipMemcpyAsync(act, act_r.data(), nb * 4, hipMemcpyHostToDevice, c.s));
    HIPCHK(p, hipStreamSynchronize(c.s));
    c.act_h = act_r;
    // start block (a caller block starts round 0 only)
    {
      dim3 grid((unsigned)(((int64_t)p->max_dof * k + 255) / 256), nb);
      if (x0 && r == 0) k_copy_start<<<grid, 256, 0, c.s>>>(c.v.meta, c.v.cls, k, vcls, x0, B[0][0]);
      else k_random_start<<<grid, 256, 0, c.s>>>(c.v.meta, c.v.cls, k, vcls,
                                                 r == 0 ? p->opts.seed : round_seed(p->opts.seed, r), B[0][0]);
      LAUNCHCHK(p);
    }
    c.use32 = mixed;
    int fp32_iters = 0;
    bool restart = false;
    rhist.clear();
    k_fill_i32<<<(nb + 255) / 256, 256, 0, c.s>>>(c.w.reached, nb, -1);
    k_fill_i32<<<(nb + 255) / 256, 256, 0, c.s>>>(c.w.xbuf, nb, -1);
    k_fill_i32<<<1, 32, 0, c.s>>>(it_dev, 1, 0);
    LAUNCHCHK(p);
    // a round that later rounds deflate against converges to tol_defl
    bool deflated_later = false;
    for (int b = 0; b < nb; ++b) deflated_later |= act_r[b] && p->meta[b].n_ev - col0 > nround;
    // columns are locked once at their round's target: below it their
    // preconditioned residuals are rounding noise that corrupts the Gram
    // matrices (the single-round target keeps a 10x margin)
    const double lock_tol = deflated_later ? tol_defl : 0.1 * p->opts.tol;
    if (images(B[0][0], B[1][0], B[2][0], B[3][0], act)) return MSGFEM_EHIP;
    if (deflate(r, 0, act)) return MSGFEM_EHIP;
    if (rr_x(act)) return MSGFEM_EHIP;
    // first half of an iteration: residual of the current Ritz block,
    // convergence, active set (boxes retired here keep X where it is)
    auto head = [&](int last) -> int {
      dim3 grid(n_chunk, nb);
      k_residual<<<grid, 1024, 0, c.s>>>(c.v.meta, c.v.cls, vcls, k, p->opts.shift, B[1][0],
                                        geneo ? B[2][0] : B[3][0], c.w.nu, B[0][1], GRAM_ROWS, n_chunk, c.w.rpart,
                                        act);
      LAUNCHCHK(p);
      k_fill_i32<<<1, 32, 0, c.s>>>(c.w.nact, 1, 0);
      // FP32 phase: residuals are estimates, no box is retired
      k_converge<<<nb, 64, 0, c.s>>>(c.v.meta, nb, k, n_chunk, c.w.rpart, c.w.nu, c.use32 ? 0.0 : p->opts.tol,
                                     c.use32 ? 0.0 : tol_defl, c.w.rho, act, c.w.iters, c.w.nact, last, status,
                                     col0, nround, it_dev, c.w.reached, buf_id(0), c.w.xbuf);
      k_add_i32<<<1, 32, 0, c.s>>>(it_dev, 1);
      LAUNCHCHK(p);
      return 0;
    };
    // second half: soft locking, preconditioned residual, images, deflation,
    // Rayleigh-Ritz over [X, W] or [X, W, P], update; the slot -> buffer map
    // rotates (X <-> Xn, P <-> Pn)
    auto tail = [&](bool hasP, int nblk) -> int {
      {
        // soft locking of converged columns (their W and P directions vanish)
        dim3 grid((unsigned)(((int64_t)p->max_dof * k + 255) / 256), nb);
        k_lock<<<grid, 256, 0, c.s>>>(c.v.meta, k, c.w.rho, lock_tol, B[0][1], hasP ? B[0][2] : nullptr,
                                      hasP ? B[1][2] : nullptr, hasP ? B[2][2] : nullptr,
                                      (hasP && !geneo) ? B[3][2] : nullptr, act);
        LAUNCHCHK(p);
      }
      // W = preconditioned residual: B2 trace of (A + s DAD)^{-1} [0; R]
      if (solve(c, 1, B[0][1], B[0][1], k, vcls, 1, act)) return MSGFEM_EHIP;
      if (images(B[0][1], B[1][1], B[2][1], B[3][1], act)) return MSGFEM_EHIP;
      if (deflate(r, 1, act)) return MSGFEM_EHIP;
      double* Zb[3] = {B[0][0], B[0][1], B[0][2]};
      double* Ab[3] = {B[1][0], B[1][1], B[1][2]};
      double* Bb[3] = {B[2][0], B[2][1], B[2][2]};
      if (gram(c, nblk, Zb, Ab, Bb, act)) return MSGFEM_EHIP;
      Blk4x3 Z;
      Out4 OX, OP;
      for (int kind = 0; kind < 4; ++kind) {
        for (int b = 0; b < 3; ++b) Z.p[kind][b] = b < nblk ? B[kind][b] : nullptr;
        OX.p[kind] = B[kind][3];
        OP.p[kind] = B[kind][4];
      }
      double by = 0, fl = 0;
      for (int b = 0; b < nb; ++b) {
        if (!c.counts(b, act)) continue;
        const BoxMeta& mt = p->meta[b];
        by += 4 * 8.0 * mt.n_dof * k * (nblk + 2);
        fl += 4 * 2 * 2.0 * mt.n_dof * (nblk * k) * k;
      }
      ProfScope ps(p, PK_UPDATE, c.s, by, fl);
      k_update<2><<<ugrid, UPD_THREADS, upd_lds(nblk * k, 2), c.s>>>(c.v.meta, nblk, k, Z, OX, OP, c.w.Y,
                                                                            c.w.Yp, act);
      LAUNCHCHK(p);
      for (int kind = 0; kind < 4; ++kind) {
        std::swap(B[kind][0], B[kind][3]);
        std::swap(B[kind][2], B[kind][4]);
      }
      return 0;
    };
    // Steady-state iterations (after the first, with P, FP64 operators) run as
    // HIP graphs of L iterations each, L the order of the slot rotation (the
    // deflation of round r swaps W with the spare slot r times), so a launch
    // leaves the slots where it found them.  The active count is read once per
    // launch; a box converged inside a launch is retired by k_converge and
    // every later kernel skips it, so the results are those of the eager loop.
    int L = 0;
    {
      int perm[5] = {0, 1, 2, 3, 4};
      for (int n = 1; n <= 12 && !L; ++n) {
        for (int q = 0; q < r; ++q) std::swap(perm[1], perm[3]);
        std::swap(perm[0], perm[3]);
        std::swap(perm[2], perm[4]);
        bool id = true;
        for (int i = 0; i < 5; ++i) id = id && perm[i] == i;
        if (id) L = n;
      }
      if (L && L < 4) L *= (4 + L - 1) / L;   // at least 4 iterations per launch
    }
    auto graph_get = [&](msgfem_plan::GraphEntry** out) -> int {
      for (auto& g : p->graphs) {
        if (g.ops == ops && g.work == work && g.status == status && g.r == r && g.pre32 == (int)c.pre32 &&
            g.L == L && g.lock_tol == lock_tol && !memcmp(g.B, B, sizeof B)) {
          *out = &g;
          return 0;
        }
      }
      if (!p->cap_stream) HIPCHK(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
      msgfem_plan::GraphEntry e{};
      e.ops = ops;
      e.work = work;
      e.status = status;
      e.r = r;
      e.pre32 = (int)c.pre32;
      e.L = L;
      e.lock_tol = lock_tol;
      memcpy(e.B, B, sizeof B);
      const hipStream_t user = c.s;
      c.s = p->cap_stream;
      HIPCHK(p, hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
      int rc = 0;
      for (int j = 0; j < L && !rc; ++j) {
        rc = head(0);
        if (!rc) rc = tail(true, 3);
      }
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(c.s, &graph);
      c.s = user;
      if (rc || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : fail(p, MSGFEM_EHIP, "LOBPCG graph capture: %s", hipGetErrorString(ec));
      }
      if (memcmp(e.B, B, sizeof B)) {
        (void)hipGraphDestroy(graph);
        return fail(p, MSGFEM_EHIP, "LOBPCG graph capture: slot rotation of order %d did not close", L);
      }
      const hipError_t ei = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return fail(p, MSGFEM_EHIP, "LOBPCG graph instantiate: %s", hipGetErrorString(ei));
      if (p->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        p->graphs.erase(p->graphs.begin());
      }
      p->graphs.push_back(e);
      *out = &p->graphs.back();
      return 0;
    };
    for (int it = 0; it <= p->opts.maxit; ++it) {
      if (use_graph && L && it >= 1 && !restart && !c.use32 && it + L <= p->opts.maxit) {
        msgfem_plan::GraphEntry* g = nullptr;
        if (graph_get(&g)) return MSGFEM_EHIP;
        HIPCHK(p, hipGraphLaunch(g->exec, c.s));
        int32_t nact_h = 0;
        HIPCHK(p, hipMemcpyAsync(&nact_h, c.w.nact, 4, hipMemcpyDeviceToHost, c.s));
        HIPCHK(p, hipStreamSynchronize(c.s));
        p->graph_launches += 1;
        p->graph_iters += L;
        it += L - 1;
        if (nact_h == 0) break;
        continue;
      }
      if (head(it == p->opts.maxit ? 1 : 0)) return MSGFEM_EHIP;
      c.act_h.resize(nb);
      HIPCHK(p, hipMemcpyAsync(c.act_h.data(), act, nb * 4, hipMemcpyDeviceToHost, c.s));
      if (c.use32) {
        rho_h.resize((size_t)nb * k);
        HIPCHK(p, hipMemcpyAsync(rho_h.data(), c.w.rho, (size_t)nb * k * 8, hipMemcpyDeviceToHost, c.s));
      }
      HIPCHK(p, hipStreamSynchronize(c.s));
      int nact = 0;
      for (int b = 0; b < nb; ++b) nact += c.act_h[b] != 0;
      if (nact == 0 || it == p->opts.maxit) break;
      if (c.use32) {
        double rmax = 0.0;
        for (int b = 0; b < nb; ++b) {
          if (!c.act_h[b]) continue;
          const int nev = std::min(nround, p->meta[b].n_ev - col0);
          for (int cc = 0; cc < nev; ++cc) rmax = std::max(rmax, rho_h[(size_t)b * k + cc]);
        }
        // leave the FP32 phase when it has done its part (rho <= switch_tol),
        // when it stagnates at the FP32 operators' accuracy (rho not halved
        // over two iterations) or at the iteration cap
        rhist.push_back(rmax);
        const size_t nh = rhist.size();
        const bool stalled = nh >= 3 && !(rhist[nh - 1] <= 0.5 * rhist[nh - 3]);
        if (!(rmax <= switch_tol) && !stalled && ++fp32_iters < fp32_cap) {
          // stay in the FP32 phase
        } else {
          c.use32 = false;
          const int64_t n = p->dofs_total * k;
          k_keep_classes<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, c.s>>>(c.v.cls, vcls, k, n,
                                                                                               B[0][0]);
          LAUNCHCHK(p);
          if (images(B[0][0], B[1][0], B[2][0], B[3][0], act)) return MSGFEM_EHIP;
          if (deflate(r, 0, act)) return MSGFEM_EHIP;
          if (rr_x(act)) return MSGFEM_EHIP;
          restart = true;
          continue;
        }
      }
      const bool hasP = it > 0 && !restart;
      const int nblk = hasP ? 3 : 2;
      restart = false;
      if (tail(hasP, nblk)) return MSGFEM_EHIP;
    }
    // this round's pairs (k_converge has set bit 1 on the boxes still active
    // after maxit); its converged block is kept for the later rounds
    HIPCHK(p, hipMemcpyAsync(act, act_r.data(), nb * 4, hipMemcpyHostToDevice, c.s));
    const XLoc xl{c.w.vec, VT, buf_id(0), c.w.xbuf};
    k_output<<<nb, 1024, 0, c.s>>>(c.v.meta, k, p->opts.shift, xl, c.w.nu, c.w.rho, evals, evecs, resid, act, col0,
                                  nround);
    LAUNCHCHK(p);
    if (r + 1 < p->rounds) {
      dim3 grid((unsigned)std::min<int64_t>(((int64_t)p->max_dof * k + 255) / 256, 4096), nb);
      for (int kind = 0; kind < nkinds; ++kind)
        k_keep_cols<<<grid, 256, 0, c.s>>>(c.v.meta, k, col0, nround, xl, kind, Yblk(r, kind));
      LAUNCHCHK(p);
    }
    HIPCHK(p, hipStreamSynchronize(c.s));   // act_r is read by the copy above
  }
  if (mask)
    k_copy_masked_i32<<<(nb + 255) / 256, 256, 0, c.s>>>(nb, mask, c.w.iters, iters);
  else
    HIPCHK(p, hipMemcpyAsync(iters, c.w.iters, nb * 4, hipMemcpyDeviceToDevice, c.s));
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_local_eigs(msgfem_plan* p, const void* ops, void* work, const double* x0,
                                 double* evals, double* evecs, double* resid, int32_t* iters,
                                 int32_t* status, void* stream) {
  return local_eigs_impl(p, ops, work, x0, nullptr, evals, evecs, resid, iters, status, stream);
}

extern "C" int msgfem_local_eigs_subset(msgfem_plan* p, const void* ops, void* work, const double* x0,
                                        const int32_t* mask, double* evals, double* evecs, double* resid,
                                        int32_t* iters, int32_t* status, void* stream) {
  if (!mask) return fail(p, MSGFEM_EARG, "null mask");
  return local_eigs_impl(p, ops, work, x0, mask, evals, evecs, resid, iters, status, stream);
}

// The operator products and solves of msgfem_local_apply with caller-chosen
// scratch: xm (dofs_total * k doubles, ops 0 and 1) and scr (the solves' w rows).
static int apply_impl(Ctx& c, int32_t op, int32_t kk, const double* x, double* y, double* xm) {
  msgfem_plan* p = c.p;
  if (op == 0 || op == 1) {
    // B3 columns are removed from A: clear the caller's block there first
    const int64_t n = p->dofs_total * kk;
    k_mask_b3<<<(unsigned)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, c.s>>>(c.v.cls, x, kk, n, xm);
    LAUNCHCHK(p);
    if (op == 0) return spmm(c, xm, y, nullptr, kk, (1 << 1) | (1 << 2), 1.0, nullptr) ? MSGFEM_EHIP : 0;
    return spmm(c, xm, nullptr, y, kk, 0, 1.0, nullptr) ? MSGFEM_EHIP : 0;
  }
  if (op == 2) return solve(c, 0, x, y, kk, 1 << 1, 1, nullptr) ? MSGFEM_EHIP : 0;
  return solve(c, 1, x, y, kk, (1 << 1) | (1 << 2), 1, nullptr) ? MSGFEM_EHIP : 0;
}

extern "C" int msgfem_local_apply(msgfem_plan* p, const void* ops, void* work, int32_t op, int32_t kk,
                                  const double* x, double* y, void* stream) {
  if (!p || !ops || !x || !y || x == y) return fail(p, MSGFEM_EARG, "bad argument");
  if (kk != p->k) return fail(p, MSGFEM_EARG, "k must equal the plan's block width %d", p->k);
  if (op < 0 || op > 3) return fail(p, MSGFEM_EARG, "unknown op %d", op);
  if (!work) return fail(p, MSGFEM_EARG, "null work buffer");
  if (set_device(p)) return MSGFEM_EHIP;
  Ctx c;
  c.p = p;
  c.v = ops_view(p, ops);
  c.s = (hipStream_t)stream;
  c.nb = (int)p->meta.size();
  c.k = p->k;
  c.w = work_view(p, work);
  return apply_impl(c, op, kk, x, y, c.w.vec + (int64_t)20 * p->vec_total);
}

// ---------------------------------------------------------------------------
// msgfem_local_apply_static: the same products and solves with the scratch in
// a file-scope device array instead of the caller's work buffer.  Host code
// never passes the array's name to a kernel (on the host it only names the
// symbol): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in g_scratch_ptr.

#define MSGFEM_STATIC_SCRATCH_MAX ((int64_t)16 << 20)
static __device__ __align__(256) unsigned char scratch[MSGFEM_STATIC_SCRATCH_MAX];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // per device ordinal, nullptr until looked up

static int static_scratch(msgfem_plan* p, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const int dev = p->device;
  if (dev < 0) return fail(p, MSGFEM_EARG, "bad device %d", dev);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(p, MSGFEM_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MSGFEM_OK;
}

// bytes of static scratch an op of this plan needs (256-aligned pieces)
static int64_t static_scratch_w_bytes(const msgfem_plan* p) {
  const int nchunk = 2 * ((p->k + 15) / 16);   // 8-column chunks, whole chunks of 16
  return align256((int64_t)2 * p->meta.size() * nchunk * p->scr_stride * 8);
}
static int64_t static_scratch_bytes(const msgfem_plan* p, int op) {
  if (op == 0 || op == 1) return align256(p->dofs_total * p->k * 8);
  const int nchunk = 2 * ((p->k + 15) / 16);
  const bool split = p->any_split[op == 2 ? 0 : 1];
  return static_scratch_w_bytes(p) + (split ? align256((int64_t)p->meta.size() * nchunk * 4 * p->sep_q * 8) : 0);
}

extern "C" int64_t msgfem_static_scratch_max(void) { return MSGFEM_STATIC_SCRATCH_MAX; }

extern "C" int msgfem_local_apply_static(msgfem_plan* p, const void* ops, int32_t op, int32_t kk, const double* x,
                                         double* y, void* stream) {
  if (!p || !ops || !x || !y || x == y) return fail(p, MSGFEM_EARG, "bad argument");
  if (kk != p->k) return fail(p, MSGFEM_EARG, "k must equal the plan's block width %d", p->k);
  if (op < 0 || op > 3) return fail(p, MSGFEM_EARG, "unknown op %d", op);
  const int64_t need = static_scratch_bytes(p, op);
  if (need > MSGFEM_STATIC_SCRATCH_MAX)
    return fail(p, MSGFEM_ESIZE,
                "op %d of this plan needs %lld bytes of scratch, more than the %lld of the static buffer "
                "(use msgfem_local_apply with a work buffer)",
                op, (long long)need, (long long)MSGFEM_STATIC_SCRATCH_MAX);
  if (set_device(p)) return MSGFEM_EHIP;
  void* base = nullptr;
  if (int rc = static_scratch(p, &base)) return rc;
  Ctx c;
  c.p = p;
  c.v = ops_view(p, ops);
  c.s = (hipStream_t)stream;
  c.nb = (int)p->meta.size();
  c.k = p->k;
  c.no_alloc = true;
  std::memset(&c.w, 0, sizeof c.w);
  // the solves' w rows and separator exchange (written before they are read)
  c.w.scr = (double*)base;
  c.w.sep = (double*)((char*)base + static_scratch_w_bytes(p));
  return apply_impl(c, op, kk, x, y, (double*)base);
}

extern "C" int msgfem_profile(msgfem_plan* p, int32_t enable) {
  if (!p) return MSGFEM_EARG;
  if (enable) {
    for (auto& r : p->prof_pending) { p->ev_pool.push_back(r.b); p->ev_pool.push_back(r.e); }
    p->prof_pending.clear();
    for (int i = 0; i < PK_N; ++i) {
      p->prof_ms[i] = p->prof_bytes[i] = p->prof_flops[i] = 0.0;
      p->prof_launches[i] = 0;
    }
  }
  p->prof_on = enable != 0;
  return MSGFEM_OK;
}

extern "C" int msgfem_plan_set_option(msgfem_plan* p, int32_t key, int64_t value) {
  if (!p) return MSGFEM_EARG;
  switch (key) {
    case MSGFEM_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(p, MSGFEM_EARG, "MSGFEM_OPT_GRAPH takes 0 or 1, not %lld",
                                               (long long)value);
      p->graph_mode = (int)value;
      if (!value) {
        for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
        p->graphs.clear();
      }
      return MSGFEM_OK;
    case MSGFEM_OPT_SPLIT: {
      if (value != 0 && value != 1) return fail(p, MSGFEM_EARG, "MSGFEM_OPT_SPLIT takes 0 or 1, not %lld",
                                               (long long)value);
      if (p->split == (int)value) return MSGFEM_OK;
      p->split = (int)value;
      for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
      p->graphs.clear();
      return plan_layout(p, p->nsd, p->mesh.n_mat);
    }
    case MSGFEM_OPT_SOLVE:
      if (value < 0 || value > 3) return fail(p, MSGFEM_EARG, "MSGFEM_OPT_SOLVE takes 0 .. 3, not %lld",
                                             (long long)value);
      p->solve_pref = (int)value;
      for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
      p->graphs.clear();
      return MSGFEM_OK;
    case MSGFEM_OPT_SPMM:
      if (value < 0 || value > 2) return fail(p, MSGFEM_EARG, "MSGFEM_OPT_SPMM takes 0 .. 2, not %lld",
                                             (long long)value);
      p->spmm_pref = (int)value;
      for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
      p->graphs.clear();
      return MSGFEM_OK;
    case MSGFEM_OPT_CHOL:
      if (value < 0 || value > 2) return fail(p, MSGFEM_EARG, "MSGFEM_OPT_CHOL takes 0 .. 2, not %lld",
                                             (long long)value);
      p->chol_pref = (int)value;
      return MSGFEM_OK;
    default:
      return fail(p, MSGFEM_EARG, "unknown plan option %d", key);
  }
}

extern "C" int msgfem_plan_get_option(const msgfem_plan* p, int32_t key, int64_t* value) {
  if (!p || !value) return MSGFEM_EARG;
  switch (key) {
    case MSGFEM_OPT_GRAPH: *value = p->graph_mode; return MSGFEM_OK;
    case MSGFEM_OPT_SPLIT: *value = p->split; return MSGFEM_OK;
    case MSGFEM_OPT_SOLVE: *value = p->solve_pref; return MSGFEM_OK;
    case MSGFEM_OPT_SPMM: *value = p->spmm_pref; return MSGFEM_OK;
    case MSGFEM_OPT_CHOL: *value = p->chol_pref; return MSGFEM_OK;
    case MSGFEM_INFO_MAX_BT_A11: *value = p->max_bt_kind[0]; return MSGFEM_OK;
    case MSGFEM_INFO_MAX_BT_AHAT: *value = p->max_bt_kind[1]; return MSGFEM_OK;
    case MSGFEM_INFO_SOLVE_FAMILY:
      *value = (solve4_kind(p, 0) ? (wide_kind(p, 0) ? 3 : 2) : 1) + 4 * (solve4_kind(p, 1) ? (wide_kind(p, 1) ? 3 : 2) : 1);
      return MSGFEM_OK;
    case MSGFEM_INFO_SPLIT_BOXES: {
      int64_t n = 0;
      for (auto& m : p->meta) n += m.nd[0] + 2 * m.nd[1];
      *value = n;
      return MSGFEM_OK;
    }
    case MSGFEM_INFO_GRAPH_LAUNCHES: *value = p->graph_launches; return MSGFEM_OK;
    case MSGFEM_INFO_GRAPH_ITERS: *value = p->graph_iters; return MSGFEM_OK;
    case MSGFEM_INFO_GRAPHS_CACHED: *value = (int64_t)p->graphs.size(); return MSGFEM_OK;
    default: return fail(const_cast<msgfem_plan*>(p), MSGFEM_EARG, "unknown plan option %d", key);
  }
}

extern "C" int msgfem_profile_stats(msgfem_plan* p, msgfem_kernel_stat* out, int32_t max_out,
                                    int32_t* n_out) {
  if (!p || !n_out) return MSGFEM_EARG;
  for (auto& r : p->prof_pending) {
    HIPCHK(p, hipEventSynchronize(r.e));
    float ms = 0.f;
    HIPCHK(p, hipEventElapsedTime(&ms, r.b, r.e));
    p->prof_ms[r.kernel] += ms;
    p->prof_bytes[r.kernel] += r.bytes;
    p->prof_flops[r.kernel] += r.flops;
    p->prof_launches[r.kernel] += 1;
    p->ev_pool.push_back(r.b);
    p->ev_pool.push_back(r.e);
  }
  p->prof_pending.clear();
  int n = 0;
  for (int i = 0; i < PK_N; ++i) {
    if (!p->prof_launches[i]) continue;
    if (out && n < max_out) {
      std::memset(&out[n], 0, sizeof(msgfem_kernel_stat));
      std::strncpy(out[n].name, PROF_NAMES[i], sizeof(out[n].name) - 1);
      out[n].launches = p->prof_launches[i];
      out[n].ms = p->prof_ms[i];
      out[n].bytes = p->prof_bytes[i];
      out[n].flops = p->prof_flops[i];
    }
    ++n;
  }
  *n_out = n;
  return MSGFEM_OK;
}

// ---------------------------------------------------------------------------
// Coarse problem

static int coarse_plan(msgfem_plan* p) {
  if (p->coarse_ready) return MSGFEM_OK;
  const int nb = (int)p->meta.size();
  if (nb != p->nsd) return fail(p, MSGFEM_EARG, "the coarse problem needs every subdomain in the batch");
  std::vector<int> seen(p->nsd, 0);
  for (auto& m : p->meta) seen[m.sd]++;
  for (int j = 0; j < p->nsd; ++j)
    if (seen[j] != 1) return fail(p, MSGFEM_EARG, "batch must list each subdomain once");
  p->row_off.assign(nb, 0);
  int NH = 0;
  for (int b = 0; b < nb; ++b) {
    p->row_off[b] = NH;
    NH += p->meta[b].n_ev;
  }
  p->NH = NH;
  p->NTc = (NH + 31) / 32;
  p->pairs.clear();
  p->pair_start.assign(nb + 1, 0);
  for (int i = 0; i < nb; ++i) {
    p->pair_start[i] = (int)p->pairs.size();
    const BoxMeta& bi = p->meta[i];
    for (int j = 0; j < nb; ++j) {
      const BoxMeta& bj = p->meta[j];
      CoarsePair pr;
      bool ok = true;
      for (int d = 0; d < 3; ++d) {
        int jlo = bj.g0[d], jhi = bj.g0[d] + (d == 0 ? bj.mx : d == 1 ? bj.my : bj.mz) - 1;
        pr.lo[d] = std::max(bi.olo[d], jlo);
        pr.hi[d] = std::min(bi.ohi[d], jhi);
        if (pr.lo[d] > pr.hi[d]) ok = false;
      }
      if (!ok) continue;
      pr.i = i;
      pr.j = j;
      pr.row_off = p->row_off[i];
      pr.col_off = p->row_off[j];
      p->pairs.push_back(pr);
    }
  }
  p->pair_start[nb] = (int)p->pairs.size();
  const int64_t kv = p->kv, nd = p->dofs_total, np = (int64_t)p->pairs.size();
  int64_t off = 0;
  p->c_faces = off; off = align256(off + 6 * sizeof(FaceLoad));
  p->c_pairs = off; off = align256(off + np * sizeof(CoarsePair));
  p->c_pstart = off; off = align256(off + (nb + 1) * 4);
  p->c_roff = off; off = align256(off + nb * 4);
  p->c_mat = off; off = align256(off + sizeof(MatDesc));
  p->c_bload = off; off = align256(off + nd * 8);
  p->c_psi = off; off = align256(off + nd * 8);
  p->c_pv = off; off = align256(off + nd * 8);
  p->c_V = off; off = align256(off + nd * kv * 8);
  p->c_Vn = off; off = align256(off + nd * kv * 8);
  p->c_AV = off; off = align256(off + nd * kv * 8);
  p->c_Ap = off; off = align256(off + nd * 8);
  p->c_rpart = off; off = align256(off + np * kv * 8);
  p->c_tiles = off; off = align256(off + ((int64_t)p->NTc * p->NTc + p->NTc) * 1024 * 8);
  p->c_y = off; off = align256(off + 2 * (int64_t)p->NTc * 32 * 8);
  p->coarse_bytes = off;
  p->coarse_ready = true;
  return MSGFEM_OK;
}

extern "C" int msgfem_select_modes(msgfem_plan* p, const void* ops, const double* evals, double t,
                                   const double* evecs, double* evecs_out, int32_t* m, int32_t* status,
                                   void* stream) {
  if (!p || !ops || !evals || !evecs || !evecs_out || !m || !status) return fail(p, MSGFEM_EARG, "null argument");
  if (!(t > 0.0)) return fail(p, MSGFEM_EARG, "the threshold must be positive (got %g)", t);
  if (set_device(p)) return MSGFEM_EHIP;
  const OpsView v = ops_view(p, ops);
  const int nb = (int)p->meta.size();
  k_select_modes<<<nb, 256, 0, (hipStream_t)stream>>>(v.meta, evals, 1.0 / t, evecs, evecs_out, m, status);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_error_norms(msgfem_plan* p, const double* u_ref, const double* u, int64_t n,
                                  double* out, void* stream) {
  if (!p || !u_ref || !u || !out) return fail(p, MSGFEM_EARG, "null argument");
  const int64_t nn = (int64_t)(p->mesh.nx + 1) * (p->mesh.ny + 1) * (p->mesh.nz + 1);
  if (n != 3 * nn) return fail(p, MSGFEM_EARG, "vector length %lld, the mesh has %lld DoFs",
                               (long long)n, (long long)(3 * nn));
  if (set_device(p)) return MSGFEM_EHIP;
  k_error_norms<<<1, 1024, 0, (hipStream_t)stream>>>(mesh_dev(p), u_ref, u, out);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

static uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

extern "C" int msgfem_box_digest(msgfem_plan* p, const void* ops, uint64_t* digest, void* stream) {
  if (!p || !ops || !digest) return fail(p, MSGFEM_EARG, "null argument");
  if (set_device(p)) return MSGFEM_EHIP;
  const OpsView v = ops_view(p, ops);
  // the eigensolver options that change the computed local space (not the seed)
  uint64_t salt = 0x5eed;
  uint64_t words[7];
  memcpy(&words[0], &p->opts.shift, 8);
  memcpy(&words[1], &p->opts.tol, 8);
  words[2] = (uint64_t)(uint32_t)p->opts.maxit;
  words[3] = (uint64_t)(uint32_t)p->k;
  words[4] = (uint64_t)(uint32_t)p->opts.geneo;
  words[5] = (uint64_t)(uint32_t)p->opts.precision;
  words[6] = (uint64_t)(uint32_t)p->overlap;
  for (int q = 0; q < 7; ++q) salt = host_mix64(salt ^ words[q]);
  const int nb = (int)p->meta.size();
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* acc = (unsigned long long*)digest;
  k_fill_i32<<<(2 * nb + 255) / 256, 256, 0, s>>>((int32_t*)digest, 2 * nb, 0);
  k_box_digest<<<dim3(32, nb), 256, 0, s>>>(v.meta, v.stencil, v.mu1, v.cls, acc);
  k_box_digest_finish<<<(nb + 63) / 64, 64, 0, s>>>(v.meta, nb, salt, acc);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_merge_eigs(msgfem_plan* dst, msgfem_plan* src, const int32_t* boxes, int32_t n_boxes,
                                 const double* src_evals,
                                 const double* src_evecs, const double* src_resid, const int32_t* src_iters,
                                 double* evals, double* evecs, double* resid, int32_t* iters, void* stream) {
  if (!dst || !src || !src_evals || !src_evecs || !src_resid || !src_iters || !evals || !evecs || !resid ||
      !iters)
    return fail(dst, MSGFEM_EARG, "null argument");
  if (src->device != dst->device) return fail(dst, MSGFEM_EARG, "the two plans are on different devices");
  if (src->opts.geneo != dst->opts.geneo)
    return fail(dst, MSGFEM_EARG, "the two plans solve different eigenproblems (geneo flag)");
  const int nsrc = (int)src->meta.size();
  std::vector<int> pick;
  if (boxes) {
    if (n_boxes < 0) return fail(dst, MSGFEM_EARG, "negative box count");
    for (int i = 0; i < n_boxes; ++i) {
      if (boxes[i] < 0 || boxes[i] >= nsrc)
        return fail(dst, MSGFEM_EARG, "source box %d outside the source batch of %d", boxes[i], nsrc);
      pick.push_back(boxes[i]);
    }
  } else {
    for (int i = 0; i < nsrc; ++i) pick.push_back(i);
  }
  std::vector<int> where(dst->nsd, -1);
  for (size_t d = 0; d < dst->meta.size(); ++d) where[dst->meta[d].sd] = (int)d;
  for (int b : pick) {
    const BoxMeta& s = src->meta[b];
    if (s.sd < 0 || s.sd >= dst->nsd || where[s.sd] < 0)
      return fail(dst, MSGFEM_EARG, "subdomain %d of the source batch is not in this plan's batch", s.sd);
    const BoxMeta& t = dst->meta[where[s.sd]];
    if (s.mx != t.mx || s.my != t.my || s.mz != t.mz || s.g0[0] != t.g0[0] || s.g0[1] != t.g0[1] ||
        s.g0[2] != t.g0[2] || s.n_dof != t.n_dof || s.n_ev != t.n_ev)
      return fail(dst, MSGFEM_EARG, "subdomain %d has another box or n_ev in the two plans", s.sd);
  }
  if (set_device(dst)) return MSGFEM_EHIP;
  for (int b : pick) {
    const BoxMeta& s = src->meta[b];
    const int d = where[s.sd];
    const BoxMeta& t = dst->meta[d];
    const int64_t nv = (int64_t)s.n_dof * s.n_ev;
    const int64_t grid = (std::max<int64_t>(nv, s.n_ev) + 255) / 256;
    k_copy_eigs<<<(unsigned)grid, 256, 0, (hipStream_t)stream>>>(
        s.n_ev, nv, src_evals + s.eval_off, src_evecs + s.evec_off, src_resid + s.eval_off, src_iters + b,
        evals + t.eval_off, evecs + t.evec_off, resid + t.eval_off, iters + d);
    LAUNCHCHK(dst);
  }
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_sizes(msgfem_plan* p, int64_t* coarse_bytes, int32_t* n_coarse) {
  if (!p || !coarse_bytes || !n_coarse) return MSGFEM_EARG;
  int rc = coarse_plan(p);
  if (rc) return rc;
  *coarse_bytes = p->coarse_bytes;
  *n_coarse = p->NH;
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_assemble(msgfem_plan* p, const void* ops, void* work, const msgfem_load* load,
                                      const double* evecs, void* coarse, double* AH, double* bH,
                                      int32_t* status, void* stream) {
  if (!p || !ops || !work || !evecs || !coarse || !AH || !bH || !status)
    return fail(p, MSGFEM_EARG, "null argument");
  int rc = coarse_plan(p);
  if (rc) return rc;
  if (set_device(p)) return MSGFEM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  OpsView v = ops_view(p, ops);
  char* cb = (char*)coarse;
  const int nb = (int)p->meta.size(), k = p->kv, NH = p->NH;
  // load description and pair tables
  std::vector<FaceLoad> faces;
  if (load) {
    if (load->n < 0 || load->n > 6 || (load->n > 0 && (!load->face || !load->g)))
      return fail(p, MSGFEM_EARG, "bad load description");
    for (int f = 0; f < load->n; ++f) {
      int fc = load->face[f];
      if (fc < 0 || fc > 5) return fail(p, MSGFEM_EARG, "face id %d out of range", fc);
      FaceLoad fl;
      fl.axis = fc / 2;
      fl.side = fc % 2;
      for (int c = 0; c < 3; ++c) fl.g[c] = load->g[3 * f + c];
      faces.push_back(fl);
    }
  }
  MatDesc md{p->NTc, p->NTc, 0, 0, 0, (int64_t)p->NTc * p->NTc * 1024};
  if (!faces.empty())
    HIPCHK(p, hipMemcpyAsync(cb + p->c_faces, faces.data(), faces.size() * sizeof(FaceLoad),
                             hipMemcpyHostToDevice, s));
  if (!p->pairs.empty())
    HIPCHK(p, hipMemcpyAsync(cb + p->c_pairs, p->pairs.data(), p->pairs.size() * sizeof(CoarsePair),
                             hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(cb + p->c_pstart, p->pair_start.data(), (nb + 1) * 4, hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(cb + p->c_roff, p->row_off.data(), nb * 4, hipMemcpyHostToDevice, s));
  HIPCHK(p, hipMemcpyAsync(cb + p->c_mat, &md, sizeof(MatDesc), hipMemcpyHostToDevice, s));
  HIPCHK(p, hipStreamSynchronize(s));
  double* bload = (double*)(cb + p->c_bload);
  double* psi = (double*)(cb + p->c_psi);
  double* pv = (double*)(cb + p->c_pv);
  double* V = (double*)(cb + p->c_V);
  double* Vn = (double*)(cb + p->c_Vn);
  double* AV = (double*)(cb + p->c_AV);
  double* Ap = (double*)(cb + p->c_Ap);
  double* rpart = (double*)(cb + p->c_rpart);
  MeshDev mdv = mesh_dev(p);
  Ctx c;
  c.p = p;
  c.v = v;
  c.w = work_view(p, work);
  c.s = s;
  c.nb = nb;
  c.k = k;
  // loads on the boxes and particular functions psi = A11^{-1} b on B1
  k_box_load<<<dim3((p->max_nodes + 255) / 256, nb), 256, 0, s>>>(v.meta, mdv, (const FaceLoad*)(cb + p->c_faces),
                                                                 (int)faces.size(), bload);
  LAUNCHCHK(p);
  if (solve(c, 0, bload, psi, 1, 1 << 1, 1, nullptr)) return MSGFEM_EHIP;
  // PoU-weighted bases and their CholQR2 orthonormalisation
  k_coarse_basis<<<dim3((unsigned)(((int64_t)p->max_dof * k + 255) / 256), nb), 256, 0, s>>>(
      v.meta, k, v.mu1, evecs, psi, V, pv);
  LAUNCHCHK(p);
  for (int pass = 0; pass < 2; ++pass) {
    double* Zb[1] = {V};
    Blk3 Z, A, B;
    Z.p[0] = A.p[0] = B.p[0] = V;
    Z.p[1] = Z.p[2] = A.p[1] = A.p[2] = B.p[1] = B.p[2] = nullptr;
    (void)Zb;
    gram_partials(k, p->n_gchunk, nb, s, v.meta, 1, Z, A, B, k, c.w.part, nullptr);
    k_gram_reduce<<<dim3((2 * k * k + 255) / 256, nb), 256, 0, s>>>(k, p->n_gchunk, c.w.part, c.w.G, nullptr);
    k_cholqr_coef<<<nb, 256, (size_t)(k * (k + 1) + k) * 8, s>>>(k, c.w.G, c.w.Y);
    Blk4x3 Zu;
    Out4 OX, OP;
    for (int kind = 0; kind < 4; ++kind) {
      Zu.p[kind][0] = Zu.p[kind][1] = Zu.p[kind][2] = nullptr;
      OX.p[kind] = OP.p[kind] = nullptr;
    }
    Zu.p[0][0] = V;
    OX.p[0] = Vn;
    auto upd = k <= 32 ? k_update<2> : k_update<6>;
    upd<<<dim3((unsigned)((p->max_dof + UPD_ROWS - 1) / UPD_ROWS), nb, 1), UPD_THREADS, upd_lds(k, k <= 32 ? 2 : 6), s>>>(
        v.meta, 1, k, Zu, OX, OP, c.w.Y, c.w.Yp, nullptr);
    LAUNCHCHK(p);
    std::swap(V, Vn);
  }
  // A V_j and A (mu_j psi_j) on the boxes (B3 rows removed)
  if (spmm(c, V, AV, nullptr, k, (1 << 1) | (1 << 2), 1.0, nullptr)) return MSGFEM_EHIP;
  if (spmm(c, pv, Ap, nullptr, 1, (1 << 1) | (1 << 2), 1.0, nullptr)) return MSGFEM_EHIP;
  // Galerkin blocks and right-hand side
  k_fill_f64<<<1024, 256, 0, s>>>(AH, (int64_t)NH * NH, 0.0);
  if (!p->pairs.empty())
    k_coarse_pairs<<<(unsigned)p->pairs.size(), 256, 0, s>>>(v.meta, (const CoarsePair*)(cb + p->c_pairs), k, V, AV,
                                                            Ap, NH, k, AH, rpart);
  k_coarse_rhs<<<nb, 256, 0, s>>>(v.meta, k, V, bload, (const int32_t*)(cb + p->c_pstart),
                                  (const int32_t*)(cb + p->c_roff), NH, k, rpart, AH, bH);
  LAUNCHCHK(p);
  (void)status;
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_solve(msgfem_plan* p, const void* ops, void* work, void* coarse,
                                   const double* AH, const double* bH, double* cvec, double* uG,
                                   double* up, int32_t* status, void* stream) {
  if (!p || !ops || !coarse || !AH || !bH || !cvec || !uG || !status)
    return fail(p, MSGFEM_EARG, "null argument");
  if (!p->coarse_ready) return fail(p, MSGFEM_EARG, "msgfem_coarse_assemble first");
  if (set_device(p)) return MSGFEM_EHIP;
  (void)work;
  hipStream_t s = (hipStream_t)stream;
  OpsView v = ops_view(p, ops);
  char* cb = (char*)coarse;
  const int NT = p->NTc, NH = p->NH, k = p->kv;
  double* tiles = (double*)(cb + p->c_tiles);
  k_fill_i32<<<1, 32, 0, s>>>(status, 1, 0);
  k_dense_tiles<<<2048, 256, 0, s>>>(AH, NH, NT, tiles);
  LAUNCHCHK(p);
  if (tile_cholesky(p, (const MatDesc*)(cb + p->c_mat), 1, NT, NT, tiles, status, s)) return MSGFEM_EHIP;
  double* ysc = (double*)(cb + p->c_y);
  double* xsc = ysc + (int64_t)NT * 32;
  if (tile_trsv(tiles, NT, NH, bH, ysc, xsc, s)) return fail(p, MSGFEM_EHIP, "coarse triangular solve launch failed");
  HIPCHK(p, hipMemcpyAsync(cvec, xsc, (size_t)NH * 8, hipMemcpyDeviceToDevice, s));
  // u^G = u^p + V c on the global mesh
  const int64_t ng = 3 * p->n_nodes_global;
  k_fill_f64<<<1024, 256, 0, s>>>(uG, ng, 0.0);
  if (up) k_fill_f64<<<1024, 256, 0, s>>>(up, ng, 0.0);
  k_prolong<<<dim3((p->max_dof + 255) / 256, (unsigned)p->meta.size()), 256, 0, s>>>(
      v.meta, mesh_dev(p), k, (const double*)(cb + p->c_V), (const double*)(cb + p->c_pv), cvec,
      (const int32_t*)(cb + p->c_roff), uG, up);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

// ---------------------------------------------------------------------------
// GenEO two-level additive Schwarz PCG (comparison solver)

namespace {
struct PcgLayout {
  int64_t meta, stencil, cls, mu, b, x, r, z, p, q, rb, zb, zero, part, sc, total;
};
}  // namespace

static PcgLayout pcg_layout(const msgfem_plan* p) {
  PcgLayout L;
  const int64_t ng = p->n_nodes_global, nd = 3 * ng, nbd = p->dofs_total;
  int64_t off = 0;
  L.meta = off; off = align256(off + sizeof(BoxMeta));
  L.stencil = off; off = align256(off + ng * 243 * 8);
  L.cls = off; off = align256(off + nd);
  L.mu = off; off = align256(off + nd * 8);
  L.b = off; off = align256(off + nd * 8);
  L.x = off; off = align256(off + nd * 8);
  L.r = off; off = align256(off + nd * 8);
  L.z = off; off = align256(off + nd * 8);
  L.p = off; off = align256(off + nd * 8);
  L.q = off; off = align256(off + nd * 8);
  L.rb = off; off = align256(off + nbd * 8);
  L.zb = off; off = align256(off + nbd * 8);
  L.zero = off; off = align256(off + nbd * 8);
  L.part = off; off = align256(off + 1024 * 8);
  L.sc = off; off = align256(off + 16 * 8);
  L.total = off;
  return L;
}

extern "C" int msgfem_pcg_sizes(msgfem_plan* p, int64_t* bytes) {
  if (!p || !bytes) return MSGFEM_EARG;
  *bytes = pcg_layout(p).total;
  return MSGFEM_OK;
}

extern "C" int msgfem_geneo_pcg(msgfem_plan* p, const void* ops, void* work, void* coarse, const double* AH,
                                const msgfem_load* load, double rtol, int32_t maxit, void* pcg, double* u,
                                int32_t* iters, double* relres, int32_t* status, void* stream) {
  if (!p || !ops || !work || !coarse || !AH || !pcg || !u || !iters || !relres || !status)
    return fail(p, MSGFEM_EARG, "null argument");
  if (!p->opts.geneo) return fail(p, MSGFEM_EARG, "msgfem_geneo_pcg needs a GenEO plan (opts.geneo = 1)");
  if (!p->coarse_ready) return fail(p, MSGFEM_EARG, "msgfem_coarse_assemble first");
  if (!(rtol > 0) || maxit < 1) return fail(p, MSGFEM_EARG, "bad rtol / maxit");
  if (set_device(p)) return MSGFEM_EHIP;
  hipStream_t s = (hipStream_t)stream;
  OpsView v = ops_view(p, ops);
  char* cb = (char*)coarse;
  char* pb = (char*)pcg;
  const PcgLayout L = pcg_layout(p);
  const int nb = (int)p->meta.size(), k = p->kv, NT = p->NTc, NH = p->NH;
  const int64_t ng = p->n_nodes_global, nd = 3 * ng;
  MeshDev md = mesh_dev(p);
  // whole-mesh box: stencil, classes (B1 free, B3 clamped), zero PoU
  BoxMeta gm;
  std::memset(&gm, 0, sizeof gm);
  gm.sd = -1;
  gm.mx = p->mesh.nx + 1; gm.my = p->mesh.ny + 1; gm.mz = p->mesh.nz + 1;
  for (int d = 0; d < 3; ++d) { gm.olo[d] = 1; gm.ohi[d] = 0; }
  gm.n_nodes = (int32_t)ng;
  gm.n_dof = (int32_t)nd;
  HIPCHK(p, hipMemcpyAsync(pb + L.meta, &gm, sizeof gm, hipMemcpyHostToDevice, s));
  std::vector<FaceLoad> faces;
  if (load) {
    if (load->n < 0 || load->n > 6 || (load->n > 0 && (!load->face || !load->g)))
      return fail(p, MSGFEM_EARG, "bad load description");
    for (int f = 0; f < load->n; ++f) {
      FaceLoad fl;
      fl.axis = load->face[f] / 2;
      fl.side = load->face[f] % 2;
      for (int c = 0; c < 3; ++c) fl.g[c] = load->g[3 * f + c];
      faces.push_back(fl);
    }
    if (!faces.empty())
      HIPCHK(p, hipMemcpyAsync(cb + p->c_faces, faces.data(), faces.size() * sizeof(FaceLoad),
                               hipMemcpyHostToDevice, s));
  }
  HIPCHK(p, hipStreamSynchronize(s));
  const BoxMeta* gmeta = (const BoxMeta*)(pb + L.meta);
  double* gst = (double*)(pb + L.stencil);
  uint8_t* gcls = (uint8_t*)(pb + L.cls);
  double* gmu = (double*)(pb + L.mu);
  double *b = (double*)(pb + L.b), *x = (double*)(pb + L.x), *r = (double*)(pb + L.r),
         *z = (double*)(pb + L.z), *pp = (double*)(pb + L.p), *q = (double*)(pb + L.q);
  double *rb = (double*)(pb + L.rb), *zb = (double*)(pb + L.zb), *zero = (double*)(pb + L.zero);
  double *part = (double*)(pb + L.part), *sc = (double*)(pb + L.sc);
  k_fill_i32<<<1, 32, 0, s>>>(status, 1, 0);
  k_assemble<<<dim3((unsigned)((ng + 3) / 4), 1), 256, 0, s>>>(gmeta, md, v.ctab, gst);
  k_classes_mu<<<dim3((unsigned)((ng + 255) / 256), 1), 256, 0, s>>>(gmeta, md, 2 * p->overlap, v.wtot, gcls, gmu);
  k_box_load<<<dim3((unsigned)((ng + 255) / 256), 1), 256, 0, s>>>(gmeta, md, (const FaceLoad*)(cb + p->c_faces),
                                                                  (int)faces.size(), b);
  k_fill_f64<<<1024, 256, 0, s>>>(zero, p->dofs_total, 0.0);
  LAUNCHCHK(p);
  // coarse factor A_0
  double* tiles = (double*)(cb + p->c_tiles);
  k_dense_tiles<<<2048, 256, 0, s>>>(AH, NH, NT, tiles);
  if (tile_cholesky(p, (const MatDesc*)(cb + p->c_mat), 1, NT, NT, tiles, status, s)) return MSGFEM_EHIP;
  double* ysc = (double*)(cb + p->c_y);
  double* xsc = ysc + (int64_t)NT * 32;
  double* rc = (double*)(cb + p->c_rpart);   // the coarse restriction (N_H <= 32 * pairs)
  Ctx c;
  c.p = p;
  c.v = v;
  c.w = work_view(p, work);
  c.s = s;
  c.nb = nb;
  c.k = k;
  const unsigned gblk = (unsigned)std::min<int64_t>((nd + 255) / 256, 2048);
  auto gspmv = [&](const double* in, double* out) -> int {
    const int gb = (int)((ng + 255) / 256);
    k_spmm<false, 1><<<dim3((unsigned)gb), 256, 0, s>>>(gmeta, 1, gb, (const double*)gst, gcls, gmu, in, out,
                                                        nullptr, 1, 1 << 1, 1.0, nullptr);
    LAUNCHCHK(p);
    return 0;
  };
  auto dot = [&](const double* a_, const double* b_, double* out) {
    k_dot_partial<<<1024, 256, 0, s>>>(a_, b_, gcls, nd, part);
    k_dot_final<<<1, 256, 0, s>>>(part, 1024, out);
  };
  auto precond = [&](const double* rin, double* zout) -> int {
    k_fill_f64<<<1024, 256, 0, s>>>(zout, nd, 0.0);
    k_gather_boxes<<<dim3((p->max_dof + 255) / 256, nb), 256, 0, s>>>(v.meta, md, v.cls, rin, rb);
    if (solve(c, 0, rb, zb, 1, 1 << 1, 1, nullptr)) return MSGFEM_EHIP;
    k_scatter_boxes<<<dim3((p->max_dof + 255) / 256, nb), 256, 0, s>>>(v.meta, md, v.cls, zb, zout);
    k_coarse_restrict<<<nb, 256, 0, s>>>(v.meta, k, (const double*)(cb + p->c_V), rb,
                                         (const int32_t*)(cb + p->c_roff), rc);
    if (tile_trsv(tiles, NT, NH, rc, ysc, xsc, s)) return MSGFEM_EHIP;
    k_prolong<<<dim3((p->max_dof + 255) / 256, nb), 256, 0, s>>>(v.meta, md, k, (const double*)(cb + p->c_V), zero,
                                                                 xsc, (const int32_t*)(cb + p->c_roff), zout,
                                                                 nullptr);
    LAUNCHCHK(p);
    return 0;
  };
  // initial residual
  HIPCHK(p, hipMemcpyAsync(x, u, nd * 8, hipMemcpyDeviceToDevice, s));
  if (gspmv(x, q)) return MSGFEM_EHIP;
  k_sub<<<gblk, 256, 0, s>>>(gcls, nd, b, q, r);
  if (precond(r, z)) return MSGFEM_EHIP;
  k_pcg_p<<<gblk, 256, 0, s>>>(gcls, nd, nullptr, z, pp);
  dot(r, z, sc + 0);
  dot(b, b, sc + 6);
  dot(r, r, sc + 3);
  double h[8];
  HIPCHK(p, hipMemcpyAsync(h, sc, 8 * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(p, hipStreamSynchronize(s));
  const double nb2 = h[6] > 0 ? std::sqrt(h[6]) : 1.0;
  double rel = std::sqrt(h[3]) / nb2;
  int it = 0;
  while (rel > rtol && it < maxit) {
    if (gspmv(pp, q)) return MSGFEM_EHIP;
    dot(pp, q, sc + 1);
    k_pcg_alpha<<<1, 1, 0, s>>>(sc);
    k_pcg_xr<<<gblk, 256, 0, s>>>(gcls, nd, sc, pp, q, x, r);
    dot(r, r, sc + 3);
    if (precond(r, z)) return MSGFEM_EHIP;
    dot(r, z, sc + 2);
    k_pcg_beta<<<1, 1, 0, s>>>(sc);
    k_pcg_p<<<gblk, 256, 0, s>>>(gcls, nd, sc, z, pp);
    LAUNCHCHK(p);
    HIPCHK(p, hipMemcpyAsync(h, sc, 8 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    rel = std::sqrt(h[3]) / nb2;
    ++it;
  }
  HIPCHK(p, hipMemcpyAsync(u, x, nd * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(p, hipStreamSynchronize(s));
  *iters = it;
  *relres = rel;
  if (rel > rtol) {
    k_status_or<<<1, 32, 0, s>>>(status, 1, 1);
    LAUNCHCHK(p);
    HIPCHK(p, hipStreamSynchronize(s));
  }
  return MSGFEM_OK;
}

// ---------------------------------------------------------------------------
// Coarse problem gathered from several plans (the local stage streamed
// through plans that hold only part of the subdomains at a time)

struct msgfem_coarse {
  int device = 0;
  msgfem_mesh mesh{};
  int nsd = 0, overlap = 0, geneo = 0, kc = 0, NH = 0, NTc = 0;
  int64_t n_nodes_global = 0, dofs_total = 0, loc_total = 0;
  int max_dof = 0, max_nt11 = 0, max_bt11 = 0;
  bool split11 = false;             // some A11 band is split (its local solve takes three phases)
  int max_nts = 0;
  bool loc_solve4 = false;          // layout of the exported local solves (GenEO): matrix-core
  bool loc_wide = false;            // ... with 16 columns per workgroup
  std::vector<int32_t> omega;       // [nsd][6] node boxes of Omega_j
  std::vector<int32_t> cores, ovs;
  std::vector<BoxMeta> meta;        // every subdomain, in subdomain order
  std::vector<CoarsePair> pairs;
  std::vector<int32_t> pair_start, row_off;
  std::vector<uint8_t> added;
  int64_t s_meta = 0, s_pairs = 0, s_pstart = 0, s_roff = 0, s_mat = 0, s_faces = 0, s_cls = 0, s_V = 0, s_AV = 0,
          s_pv = 0, s_Ap = 0, s_bload = 0, s_rpart = 0, s_rc = 0, s_tiles = 0, s_y = 0, s_loc = 0, store_bytes = 0;
  std::string err;
};

static int cfail(msgfem_coarse* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define CHIPCHK(c, call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return cfail(c, MSGFEM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define CLAUNCHCHK(c)                                                                      \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess)                                                                  \
      return cfail(c, MSGFEM_EHIP, "launch failed (line %d): %s", __LINE__, hipGetErrorString(e_)); \
  } while (0)

extern "C" int msgfem_coarse_create(msgfem_coarse** out, int device, const msgfem_mesh* mesh,
                                    const msgfem_decomp* dec, const int32_t* n_ev, int32_t geneo) {
  if (!out || !mesh || !dec || !n_ev) return MSGFEM_EARG;
  msgfem_coarse* c = new msgfem_coarse();
  *out = c;
  c->device = device;
  c->mesh = *mesh;
  c->nsd = dec->nsd;
  c->overlap = dec->overlap;
  c->geneo = geneo != 0;
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || mesh->n_mat < 1) return cfail(c, MSGFEM_EARG, "bad mesh dimensions");
  if (dec->nsd < 1 || !dec->cores || !dec->ovs || dec->overlap < 1)
    return cfail(c, MSGFEM_EARG, "bad decomposition (nsd >= 1, overlap >= 1 required)");
  const int N[3] = {mesh->nx, mesh->ny, mesh->nz};
  c->n_nodes_global = (int64_t)(N[0] + 1) * (N[1] + 1) * (N[2] + 1);
  c->cores.assign(dec->cores, dec->cores + 6 * (size_t)dec->nsd);
  c->ovs.assign(dec->ovs, dec->ovs + dec->nsd);
  c->omega.resize(6 * (size_t)dec->nsd);
  for (int j = 0; j < dec->nsd; ++j) {
    const int32_t* cr = dec->cores + 6 * j;
    for (int d = 0; d < 3; ++d) {
      if (cr[d] < 0 || cr[3 + d] > N[d] || cr[d] >= cr[3 + d]) return cfail(c, MSGFEM_EARG, "core %d out of the mesh", j);
      c->omega[6 * j + d] = std::max(cr[d] - dec->overlap, 0);
      c->omega[6 * j + 3 + d] = std::min(cr[3 + d] + dec->overlap, N[d]);
    }
    if (dec->ovs[j] < 0) return cfail(c, MSGFEM_EARG, "ovs[%d] < 0", j);
    if (n_ev[j] < 1 || n_ev[j] > MAX_NEV)
      return cfail(c, MSGFEM_EARG, "n_ev[%d] = %d outside [1, %d]", j, n_ev[j], MAX_NEV);
  }
  c->meta.resize(dec->nsd);
  int64_t dof_off = 0, node_off = 0, loc_off = 0;
  int kc = 0;
  for (int j = 0; j < dec->nsd; ++j) {
    BoxMeta& m = c->meta[j];
    if (const char* e = box_geometry(N, dec, c->omega.data(), c->geneo, j, n_ev[j], m))
      return cfail(c, MSGFEM_EARG, "subdomain %d: %s", j, e);
    m.node_off = node_off;
    m.dof_off = dof_off;
    m.eval_off = c->NH;
    // the band parts of a plan with the default layout (MSGFEM_OPT_SPLIT = 1)
    band_parts(m, true);
    if (c->geneo) {
      for (int pi = 0; pi < (m.nd[0] ? 3 : 1); ++pi) {
        BandPart& q = m.part[0][pi];
        q.fw = loc_off;
        loc_off += solve_copy_doubles(q.NT, q.BT);
        q.bw = loc_off;
        loc_off += solve_copy_doubles(q.NT, q.BT);
        q.ioff = loc_off;            // D^{-1} tiles, compact
        loc_off += (int64_t)q.NT * MSG_TILE2;
        c->max_nt11 = std::max(c->max_nt11, q.NT);
        c->max_bt11 = std::max(c->max_bt11, q.BT);
      }
      if (m.nd[0]) {
        c->split11 = true;
        c->max_nts = std::max(c->max_nts, m.part[0][2].NT);
      }
      m.flags |= BOX_COMPACT_DINV;
    }
    node_off += m.n_nodes;
    dof_off += m.n_dof;
    c->NH += m.n_ev;
    kc = std::max(kc, m.n_ev);
    c->max_dof = std::max(c->max_dof, m.n_dof);
  }
  c->kc = kc + (kc & 1);
  c->dofs_total = dof_off;
  c->loc_total = loc_off;
  c->NTc = (c->NH + 31) / 32;
  c->loc_solve4 = c->max_bt11 - 1 <= 8 * SOLVE4_MAX_SLOTS;
  c->loc_wide = c->loc_solve4 && c->max_bt11 <= WIDE_MAX_BT;
  if (c->geneo && c->max_bt11 > SOLVE_MAX_BT)
    return cfail(c, MSGFEM_ESIZE, "band of %d tiles too wide for the block solve", c->max_bt11);
  // pairs (i, j): Omega_i meets the box of j (the support of A V_j)
  c->row_off.assign(c->nsd, 0);
  c->pair_start.assign(c->nsd + 1, 0);
  for (int i = 0; i < c->nsd; ++i) c->row_off[i] = (int)c->meta[i].eval_off;
  for (int i = 0; i < c->nsd; ++i) {
    c->pair_start[i] = (int)c->pairs.size();
    const BoxMeta& bi = c->meta[i];
    for (int j = 0; j < c->nsd; ++j) {
      const BoxMeta& bj = c->meta[j];
      CoarsePair pr;
      bool ok = true;
      for (int d = 0; d < 3; ++d) {
        int jlo = bj.g0[d], jhi = bj.g0[d] + (d == 0 ? bj.mx : d == 1 ? bj.my : bj.mz) - 1;
        pr.lo[d] = std::max(bi.olo[d], jlo);
        pr.hi[d] = std::min(bi.ohi[d], jhi);
        if (pr.lo[d] > pr.hi[d]) ok = false;
      }
      if (!ok) continue;
      pr.i = i;
      pr.j = j;
      pr.row_off = c->row_off[i];
      pr.col_off = c->row_off[j];
      c->pairs.push_back(pr);
    }
  }
  c->pair_start[c->nsd] = (int)c->pairs.size();
  c->added.assign(c->nsd, 0);
  const int64_t nd = c->dofs_total, np = (int64_t)c->pairs.size(), K = c->kc;
  int64_t off = 0;
  c->s_meta = off; off = align256(off + (int64_t)c->nsd * sizeof(BoxMeta));
  c->s_pairs = off; off = align256(off + np * sizeof(CoarsePair));
  c->s_pstart = off; off = align256(off + (c->nsd + 1) * 4);
  c->s_roff = off; off = align256(off + c->nsd * 4);
  c->s_mat = off; off = align256(off + sizeof(MatDesc));
  c->s_faces = off; off = align256(off + 6 * sizeof(FaceLoad));
  c->s_cls = off; off = align256(off + nd);
  c->s_V = off; off = align256(off + nd * K * 8);
  c->s_AV = off; off = align256(off + nd * K * 8);
  c->s_pv = off; off = align256(off + nd * 8);
  c->s_Ap = off; off = align256(off + nd * 8);
  c->s_bload = off; off = align256(off + nd * 8);
  c->s_rpart = off; off = align256(off + np * K * 8);
  c->s_rc = off; off = align256(off + (int64_t)c->NTc * 32 * 8);
  c->s_tiles = off; off = align256(off + ((int64_t)c->NTc * c->NTc + c->NTc) * 1024 * 8);
  c->s_y = off; off = align256(off + 2 * (int64_t)c->NTc * 32 * 8);
  c->s_loc = off; off = align256(off + c->loc_total * 4);
  c->store_bytes = off;
  return MSGFEM_OK;
}

extern "C" void msgfem_coarse_destroy(msgfem_coarse* c) { delete c; }

extern "C" const char* msgfem_coarse_error(const msgfem_coarse* c) { return c ? c->err.c_str() : "null coarse object"; }

extern "C" int msgfem_coarse_store_sizes(const msgfem_coarse* c, int64_t* store_bytes, int32_t* n_coarse,
                                         int32_t* n_columns) {
  if (!c || !store_bytes || !n_coarse) return MSGFEM_EARG;
  *store_bytes = c->store_bytes;
  *n_coarse = c->NH;
  if (n_columns) *n_columns = c->kc;
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_box(const msgfem_coarse* c, int32_t sd, int64_t* dof_off, int32_t* n_dof,
                                 int32_t* row_off) {
  if (!c || sd < 0 || sd >= c->nsd) return MSGFEM_EARG;
  if (dof_off) *dof_off = c->meta[sd].dof_off;
  if (n_dof) *n_dof = c->meta[sd].n_dof;
  if (row_off) *row_off = c->row_off[sd];
  return MSGFEM_OK;
}

static int coarse_upload_tables(msgfem_coarse* c, char* st, hipStream_t s) {
  CHIPCHK(c, hipMemcpyAsync(st + c->s_meta, c->meta.data(), c->meta.size() * sizeof(BoxMeta), hipMemcpyHostToDevice, s));
  if (!c->pairs.empty())
    CHIPCHK(c, hipMemcpyAsync(st + c->s_pairs, c->pairs.data(), c->pairs.size() * sizeof(CoarsePair),
                              hipMemcpyHostToDevice, s));
  CHIPCHK(c, hipMemcpyAsync(st + c->s_pstart, c->pair_start.data(), c->pair_start.size() * 4, hipMemcpyHostToDevice, s));
  CHIPCHK(c, hipMemcpyAsync(st + c->s_roff, c->row_off.data(), c->row_off.size() * 4, hipMemcpyHostToDevice, s));
  return MSGFEM_OK;
}

static int load_faces(const msgfem_load* load, std::vector<FaceLoad>& faces) {
  faces.clear();
  if (!load) return 0;
  if (load->n < 0 || load->n > 6 || (load->n > 0 && (!load->face || !load->g))) return 1;
  for (int f = 0; f < load->n; ++f) {
    const int fc = load->face[f];
    if (fc < 0 || fc > 5) return 1;
    FaceLoad fl;
    fl.axis = fc / 2;
    fl.side = fc % 2;
    for (int q = 0; q < 3; ++q) fl.g[q] = load->g[3 * f + q];
    faces.push_back(fl);
  }
  return 0;
}

extern "C" int msgfem_coarse_add(msgfem_coarse* c, msgfem_plan* p, const void* ops, void* work,
                                 const msgfem_load* load, const double* evecs, void* store, void* stream) {
  if (!c || !p || !ops || !work || !evecs || !store) return cfail(c, MSGFEM_EARG, "null argument");
  if (p->device != c->device) return cfail(c, MSGFEM_EARG, "the plan is on device %d, the coarse object on %d",
                                           p->device, c->device);
  if (p->mesh.nx != c->mesh.nx || p->mesh.ny != c->mesh.ny || p->mesh.nz != c->mesh.nz || p->nsd != c->nsd ||
      p->overlap != c->overlap || (p->opts.geneo != 0) != (c->geneo != 0))
    return cfail(c, MSGFEM_EARG, "the plan's mesh, decomposition or eigenproblem differs from the coarse object's");
  for (const BoxMeta& m : p->meta) {
    const BoxMeta& t = c->meta[m.sd];
    if (m.mx != t.mx || m.my != t.my || m.mz != t.mz || m.g0[0] != t.g0[0] || m.g0[1] != t.g0[1] ||
        m.g0[2] != t.g0[2] || m.n_ev != t.n_ev)
      return cfail(c, MSGFEM_EARG, "subdomain %d has another box or n_ev in the plan", m.sd);
    if (c->geneo && (m.nd[0] != t.nd[0] || m.part[0][0].NT != t.part[0][0].NT))
      return cfail(c, MSGFEM_EARG, "subdomain %d: the plan's interior band layout differs from the coarse object's "
                   "(the store takes the default MSGFEM_OPT_SPLIT)", m.sd);
  }
  if (c->geneo && (solve4_kind(p, 0) != c->loc_solve4 || wide_kind(p, 0) != c->loc_wide))
    return cfail(c, MSGFEM_EARG,
                 "the plan's interior factors use the %s solve layout, the coarse object the %s one (give the plan "
                 "a box with the widest band)",
                 solve4_kind(p, 0) ? "matrix-core" : "vector", c->loc_solve4 ? "matrix-core" : "vector");
  std::vector<FaceLoad> faces;
  if (load_faces(load, faces)) return cfail(c, MSGFEM_EARG, "bad load description");
  if (set_device(p)) return cfail(c, MSGFEM_EHIP, "%s", p->err.c_str());
  hipStream_t s = (hipStream_t)stream;
  char* st = (char*)store;
  if (int rc = coarse_upload_tables(c, st, s)) return rc;
  if (!faces.empty())
    CHIPCHK(c, hipMemcpyAsync(st + c->s_faces, faces.data(), faces.size() * sizeof(FaceLoad), hipMemcpyHostToDevice, s));
  // the host copies above must stay valid until the copies are done (faces is local)
  CHIPCHK(c, hipStreamSynchronize(s));
  Ctx x;
  x.p = p;
  x.v = ops_view(p, ops);
  x.w = work_view(p, work);
  x.s = s;
  x.nb = (int)p->meta.size();
  x.k = p->k;
  const int k = p->kv, nb = x.nb;
  const int64_t nd = p->dofs_total, VK = nd * k;
  double* V = x.w.vec;
  double* Vn = x.w.vec + VK;
  double* AV = x.w.vec + 2 * VK;
  double* psi = x.w.vec + 3 * VK;
  double* pv = psi + nd;
  double* Ap = psi + 2 * nd;
  double* bload = psi + 3 * nd;
  MeshDev mdv = mesh_dev(p);
  k_box_load<<<dim3((p->max_nodes + 255) / 256, nb), 256, 0, s>>>(x.v.meta, mdv, (const FaceLoad*)(st + c->s_faces),
                                                                 (int)faces.size(), bload);
  CLAUNCHCHK(c);
  if (solve(x, 0, bload, psi, 1, 1 << 1, 1, nullptr)) return cfail(c, MSGFEM_EHIP, "%s", p->err.c_str());
  k_coarse_basis<<<dim3((unsigned)(((int64_t)p->max_dof * k + 255) / 256), nb), 256, 0, s>>>(x.v.meta, k, x.v.mu1, evecs,
                                                                                          psi, V, pv);
  CLAUNCHCHK(c);
  for (int pass = 0; pass < 2; ++pass) {
    Blk3 Z, A, B;
    Z.p[0] = A.p[0] = B.p[0] = V;
    Z.p[1] = Z.p[2] = A.p[1] = A.p[2] = B.p[1] = B.p[2] = nullptr;
    gram_partials(k, p->n_gchunk, nb, s, x.v.meta, 1, Z, A, B, k, x.w.part, nullptr);
    k_gram_reduce<<<dim3((2 * k * k + 255) / 256, nb), 256, 0, s>>>(k, p->n_gchunk, x.w.part, x.w.G, nullptr);
    k_cholqr_coef<<<nb, 256, (size_t)(k * (k + 1) + k) * 8, s>>>(k, x.w.G, x.w.Y);
    Blk4x3 Zu;
    Out4 OX, OP;
    for (int kind = 0; kind < 4; ++kind) {
      Zu.p[kind][0] = Zu.p[kind][1] = Zu.p[kind][2] = nullptr;
      OX.p[kind] = OP.p[kind] = nullptr;
    }
    Zu.p[0][0] = V;
    OX.p[0] = Vn;
    auto upd = k <= 32 ? k_update<2> : k_update<6>;
    upd<<<dim3((unsigned)((p->max_dof + UPD_ROWS - 1) / UPD_ROWS), nb, 1), UPD_THREADS, upd_lds(k, k <= 32 ? 2 : 6), s>>>(
        x.v.meta, 1, k, Zu, OX, OP, x.w.Y, x.w.Yp, nullptr);
    CLAUNCHCHK(c);
    std::swap(V, Vn);
  }
  if (spmm(x, V, AV, nullptr, k, (1 << 1) | (1 << 2), 1.0, nullptr)) return cfail(c, MSGFEM_EHIP, "%s", p->err.c_str());
  if (spmm(x, pv, Ap, nullptr, 1, (1 << 1) | (1 << 2), 1.0, nullptr)) return cfail(c, MSGFEM_EHIP, "%s", p->err.c_str());
  const int K = c->kc;
  k_store_box<<<dim3((unsigned)(((int64_t)p->max_dof * K + 255) / 256), nb), 256, 0, s>>>(
      x.v.meta, (const BoxMeta*)(st + c->s_meta), k, K, V, AV, pv, Ap, bload, x.v.cls, (double*)(st + c->s_V),
      (double*)(st + c->s_AV), (double*)(st + c->s_pv), (double*)(st + c->s_Ap), (double*)(st + c->s_bload),
      (uint8_t*)(st + c->s_cls));
  CLAUNCHCHK(c);
  if (c->geneo) {
    k_store_local32<<<dim3(2048, nb), 256, 0, s>>>(x.v.meta, (const BoxMeta*)(st + c->s_meta), x.v.fac,
                                                   (float*)(st + c->s_loc));
    CLAUNCHCHK(c);
  }
  for (const BoxMeta& m : p->meta) c->added[m.sd] = 1;
  return MSGFEM_OK;
}

static int coarse_all_added(msgfem_coarse* c) {
  for (int j = 0; j < c->nsd; ++j)
    if (!c->added[j]) return cfail(c, MSGFEM_EARG, "subdomain %d has not been added to the coarse store", j);
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_galerkin(msgfem_coarse* c, void* store, double* AH, double* bH, void* stream) {
  if (!c || !store || !AH || !bH) return cfail(c, MSGFEM_EARG, "null argument");
  if (int rc = coarse_all_added(c)) return rc;
  CHIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  char* st = (char*)store;
  if (int rc = coarse_upload_tables(c, st, s)) return rc;
  const int NH = c->NH;
  k_fill_f64<<<4096, 256, 0, s>>>(AH, (int64_t)NH * NH, 0.0);
  if (!c->pairs.empty())
    k_coarse_pairs<<<(unsigned)c->pairs.size(), 256, 0, s>>>((const BoxMeta*)(st + c->s_meta),
                                                             (const CoarsePair*)(st + c->s_pairs), c->kc,
                                                             (const double*)(st + c->s_V), (const double*)(st + c->s_AV),
                                                             (const double*)(st + c->s_Ap), NH, c->kc, AH,
                                                             (double*)(st + c->s_rpart));
  k_coarse_rhs<<<c->nsd, 256, 0, s>>>((const BoxMeta*)(st + c->s_meta), c->kc, (const double*)(st + c->s_V),
                                      (const double*)(st + c->s_bload), (const int32_t*)(st + c->s_pstart),
                                      (const int32_t*)(st + c->s_roff), NH, c->kc, (const double*)(st + c->s_rpart),
                                      AH, bH);
  CLAUNCHCHK(c);
  return MSGFEM_OK;
}

// tile Cholesky of the dense coarse matrix into the store's tiles
static int coarse_factor(msgfem_coarse* c, char* st, const double* AH, int32_t* status, hipStream_t s) {
  const int NT = c->NTc;
  MatDesc md{NT, NT, 0, 0, 0, (int64_t)NT * NT * 1024};
  CHIPCHK(c, hipMemcpyAsync(st + c->s_mat, &md, sizeof md, hipMemcpyHostToDevice, s));
  CHIPCHK(c, hipStreamSynchronize(s));
  double* tiles = (double*)(st + c->s_tiles);
  k_fill_i32<<<1, 32, 0, s>>>(status, 1, 0);
  k_dense_tiles<<<4096, 256, 0, s>>>(AH, c->NH, NT, tiles);
  CLAUNCHCHK(c);
  if (tile_cholesky(nullptr, (const MatDesc*)(st + c->s_mat), 1, NT, NT, tiles, status, s))
    return cfail(c, MSGFEM_EHIP, "coarse Cholesky launch failed");
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_solve_store(msgfem_coarse* c, void* store, const double* AH, const double* bH, double* cvec,
                                         double* uG, double* up, int32_t* status, void* stream) {
  if (!c || !store || !AH || !bH || !cvec || !uG || !status) return cfail(c, MSGFEM_EARG, "null argument");
  if (int rc = coarse_all_added(c)) return rc;
  CHIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  char* st = (char*)store;
  if (int rc = coarse_upload_tables(c, st, s)) return rc;
  if (int rc = coarse_factor(c, st, AH, status, s)) return rc;
  const int NT = c->NTc;
  double* ysc = (double*)(st + c->s_y);
  double* xsc = ysc + (int64_t)NT * 32;
  if (tile_trsv((const double*)(st + c->s_tiles), NT, c->NH, bH, ysc, xsc, s))
    return cfail(c, MSGFEM_EHIP, "coarse triangular solve launch failed");
  CHIPCHK(c, hipMemcpyAsync(cvec, xsc, (size_t)c->NH * 8, hipMemcpyDeviceToDevice, s));
  const int64_t ng = 3 * c->n_nodes_global;
  k_fill_f64<<<1024, 256, 0, s>>>(uG, ng, 0.0);
  if (up) k_fill_f64<<<1024, 256, 0, s>>>(up, ng, 0.0);
  MeshDev md;
  md.nx = c->mesh.nx; md.ny = c->mesh.ny; md.nz = c->mesh.nz; md.n_mat = c->mesh.n_mat;
  md.xyz = c->mesh.node_xyz; md.elem_mat = c->mesh.elem_mat; md.materials = c->mesh.materials;
  md.dirichlet = c->mesh.dirichlet;
  k_prolong<<<dim3((c->max_dof + 255) / 256, c->nsd), 256, 0, s>>>((const BoxMeta*)(st + c->s_meta), md, c->kc,
                                                                   (const double*)(st + c->s_V),
                                                                   (const double*)(st + c->s_pv), cvec,
                                                                   (const int32_t*)(st + c->s_roff), uG, up);
  CLAUNCHCHK(c);
  return MSGFEM_OK;
}

// Block solve of kind `kind` on FP32 factor copies for a box list given only
// on the device (no plan): the store-based PCG's local Dirichlet solves.
static int solve_f32(hipStream_t s, const BoxMeta* meta, int nb, int max_bt, bool use4, bool wide, int kind,
                     const float* ft, const uint8_t* cls, const double* in, double* out, int kk, int out_classes,
                     int zero_rest, double* scr, int64_t scr_stride, bool split, double* sep, int64_t sep_q) {
  const int kc = wide ? 16 : KC;
  const int nchunk = (kk + kc - 1) / kc;
  const size_t lds = (size_t)max_bt * 32 * kc * 8;
  auto launch = [&](auto kern) {
    for (int ph = split ? 1 : 0; ph <= (split ? 3 : 0); ++ph) {
      const int nun = (ph == 1 || ph == 3) ? 2 * nb : nb;
      dim3 grid(8 * nchunk * ((nun + 7) / 8));
      kern<<<grid, 512, lds, s>>>(meta, nb, nchunk, kind, ft, cls, in, out, kk, out_classes, zero_rest, scr,
                                  scr_stride, nullptr, ph, sep, sep_q, nullptr);
    }
  };
  if (use4 && wide) {
    const int ns = solve4_nslot(max_bt);
    if (ns <= 1) launch(k_band_solve4<1, true, float>);
    else if (ns == 2) launch(k_band_solve4<2, true, float>);
    else if (ns == 3) launch(k_band_solve4<3, true, float>);
    else launch(k_band_solve4<4, true, float>);
  } else if (use4) {
    const int ns = solve4_nslot(max_bt);
    if (ns <= 1) launch(k_band_solve4<1, false, float>);
    else if (ns == 2) launch(k_band_solve4<2, false, float>);
    else if (ns == 3) launch(k_band_solve4<3, false, float>);
    else if (ns == 4) launch(k_band_solve4<4, false, float>);
    else if (ns == 5) launch(k_band_solve4<5, false, float>);
    else launch(k_band_solve4<8, false, float>);
  } else if (max_bt - 1 > SOLVE_TILES) {
    launch(k_band_solve<KC, 2, float>);
  } else {
    launch(k_band_solve<KC, 1, float>);
  }
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

namespace {
struct CPcgLayout {
  int64_t meta, ctab, omega, wtot, stencil, cls, mu, b, x, r, z, p, q, rb, zb, zero, part, sc, scr, sep, total;
  int64_t scr_stride, sep_q;
};
}  // namespace

static CPcgLayout cpcg_layout(const msgfem_coarse* c) {
  CPcgLayout L;
  const int64_t ng = c->n_nodes_global, nd = 3 * ng, nbd = c->dofs_total;
  const int kc = c->loc_wide ? 16 : KC;
  L.scr_stride = (int64_t)(c->max_nt11 + 1) * 32 * kc;
  L.sep_q = (int64_t)(c->max_nts + 1) * 32 * kc;
  int64_t off = 0;
  L.meta = off; off = align256(off + sizeof(BoxMeta));
  L.ctab = off; off = align256(off + (int64_t)c->mesh.n_mat * 36 * 8);
  L.omega = off; off = align256(off + (int64_t)c->nsd * 6 * 4);
  L.wtot = off; off = align256(off + ng * 4);
  L.stencil = off; off = align256(off + ng * 243 * 8);
  L.cls = off; off = align256(off + nd);
  L.mu = off; off = align256(off + nd * 8);
  L.b = off; off = align256(off + nd * 8);
  L.x = off; off = align256(off + nd * 8);
  L.r = off; off = align256(off + nd * 8);
  L.z = off; off = align256(off + nd * 8);
  L.p = off; off = align256(off + nd * 8);
  L.q = off; off = align256(off + nd * 8);
  L.rb = off; off = align256(off + nbd * 8);
  L.zb = off; off = align256(off + nbd * 8);
  L.zero = off; off = align256(off + nbd * 8);
  L.part = off; off = align256(off + 1024 * 8);
  L.sc = off; off = align256(off + 16 * 8);
  L.scr = off; off = align256(off + (int64_t)2 * c->nsd * L.scr_stride * 8);
  L.sep = off; off = align256(off + (c->split11 ? (int64_t)c->nsd * 4 * L.sep_q * 8 : 0));
  L.total = off;
  return L;
}

extern "C" int msgfem_coarse_pcg_sizes(const msgfem_coarse* c, int64_t* bytes) {
  if (!c || !bytes) return MSGFEM_EARG;
  *bytes = cpcg_layout(c).total;
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_pcg(msgfem_coarse* c, void* store, const double* A0, const msgfem_load* load, double rtol,
                                 int32_t maxit, void* pcg, double* u, int32_t* iters, double* relres, int32_t* status,
                                 void* stream) {
  if (!c || !store || !A0 || !pcg || !u || !iters || !relres || !status) return cfail(c, MSGFEM_EARG, "null argument");
  if (!c->geneo) return cfail(c, MSGFEM_EARG, "msgfem_coarse_pcg needs a GenEO coarse object (geneo = 1)");
  if (!(rtol > 0) || maxit < 1) return cfail(c, MSGFEM_EARG, "bad rtol / maxit");
  if (int rc = coarse_all_added(c)) return rc;
  std::vector<FaceLoad> faces;
  if (load_faces(load, faces)) return cfail(c, MSGFEM_EARG, "bad load description");
  CHIPCHK(c, hipSetDevice(c->device));
  lds_attributes();
  hipStream_t s = (hipStream_t)stream;
  char* st = (char*)store;
  char* pb = (char*)pcg;
  const CPcgLayout L = cpcg_layout(c);
  const int nsd = c->nsd, K = c->kc, NT = c->NTc, NH = c->NH;
  const int64_t ng = c->n_nodes_global, nd = 3 * ng;
  MeshDev md;
  md.nx = c->mesh.nx; md.ny = c->mesh.ny; md.nz = c->mesh.nz; md.n_mat = c->mesh.n_mat;
  md.xyz = c->mesh.node_xyz; md.elem_mat = c->mesh.elem_mat; md.materials = c->mesh.materials;
  md.dirichlet = c->mesh.dirichlet;
  // whole-mesh box: stencil, classes (B1 free, B3 clamped), zero PoU
  BoxMeta gm;
  std::memset(&gm, 0, sizeof gm);
  gm.sd = -1;
  gm.mx = c->mesh.nx + 1; gm.my = c->mesh.ny + 1; gm.mz = c->mesh.nz + 1;
  for (int d = 0; d < 3; ++d) { gm.olo[d] = 1; gm.ohi[d] = 0; }
  gm.n_nodes = (int32_t)ng;
  gm.n_dof = (int32_t)nd;
  if (int rc = coarse_upload_tables(c, st, s)) return rc;
  CHIPCHK(c, hipMemcpyAsync(pb + L.meta, &gm, sizeof gm, hipMemcpyHostToDevice, s));
  CHIPCHK(c, hipMemcpyAsync(pb + L.omega, c->omega.data(), c->omega.size() * 4, hipMemcpyHostToDevice, s));
  if (!faces.empty())
    CHIPCHK(c, hipMemcpyAsync(st + c->s_faces, faces.data(), faces.size() * sizeof(FaceLoad), hipMemcpyHostToDevice, s));
  CHIPCHK(c, hipStreamSynchronize(s));
  const BoxMeta* gmeta = (const BoxMeta*)(pb + L.meta);
  double* ctab = (double*)(pb + L.ctab);
  int32_t* wtot = (int32_t*)(pb + L.wtot);
  double* gst = (double*)(pb + L.stencil);
  uint8_t* gcls = (uint8_t*)(pb + L.cls);
  double* gmu = (double*)(pb + L.mu);
  double *b = (double*)(pb + L.b), *x = (double*)(pb + L.x), *r = (double*)(pb + L.r), *z = (double*)(pb + L.z),
         *pp = (double*)(pb + L.p), *q = (double*)(pb + L.q);
  double *rb = (double*)(pb + L.rb), *zb = (double*)(pb + L.zb), *zero = (double*)(pb + L.zero);
  double *part = (double*)(pb + L.part), *sc = (double*)(pb + L.sc), *scr = (double*)(pb + L.scr);
  const BoxMeta* smeta = (const BoxMeta*)(st + c->s_meta);
  const uint8_t* scls = (const uint8_t*)(st + c->s_cls);
  const double* sV = (const double*)(st + c->s_V);
  const int32_t* sroff = (const int32_t*)(st + c->s_roff);
  double* rc = (double*)(st + c->s_rc);
  k_materials<<<(c->mesh.n_mat + 63) / 64, 64, 0, s>>>(c->mesh.materials, c->mesh.n_mat, ctab);
  k_fill_i32<<<1024, 256, 0, s>>>(wtot, ng, 0);
  {
    int maxo = 1;
    for (int j = 0; j < nsd; ++j) {
      const int32_t* o = &c->omega[6 * j];
      maxo = std::max(maxo, (o[3] - o[0] + 1) * (o[4] - o[1] + 1) * (o[5] - o[2] + 1));
    }
    k_pou_total<<<dim3((maxo + 255) / 256, nsd), 256, 0, s>>>((const int32_t*)(pb + L.omega), nsd, c->mesh.nx,
                                                              c->mesh.ny, c->mesh.nz, 2 * c->overlap, wtot);
  }
  k_assemble<<<dim3((unsigned)((ng + 3) / 4), 1), 256, 0, s>>>(gmeta, md, ctab, gst);
  k_classes_mu<<<dim3((unsigned)((ng + 255) / 256), 1), 256, 0, s>>>(gmeta, md, 2 * c->overlap, wtot, gcls, gmu);
  k_box_load<<<dim3((unsigned)((ng + 255) / 256), 1), 256, 0, s>>>(gmeta, md, (const FaceLoad*)(st + c->s_faces),
                                                                  (int)faces.size(), b);
  k_fill_f64<<<1024, 256, 0, s>>>(zero, c->dofs_total, 0.0);
  CLAUNCHCHK(c);
  // coarse factor A_0
  if (int rc_ = coarse_factor(c, st, A0, status, s)) return rc_;
  const double* tiles = (const double*)(st + c->s_tiles);
  double* ysc = (double*)(st + c->s_y);
  double* xsc = ysc + (int64_t)NT * 32;
  const unsigned gblk = (unsigned)std::min<int64_t>((nd + 255) / 256, 4096);
  auto gspmv = [&](const double* in, double* out) {
    const int gb = (int)((ng + 255) / 256);
    k_spmm<false, 1><<<dim3((unsigned)gb), 256, 0, s>>>(gmeta, 1, gb, (const double*)gst, gcls, gmu, in, out, nullptr,
                                                        1, 1 << 1, 1.0, nullptr);
  };
  auto dot = [&](const double* a_, const double* b_, double* out) {
    k_dot_partial<<<1024, 256, 0, s>>>(a_, b_, gcls, nd, part);
    k_dot_final<<<1, 256, 0, s>>>(part, 1024, out);
  };
  auto precond = [&](const double* rin, double* zout) -> int {
    k_fill_f64<<<4096, 256, 0, s>>>(zout, nd, 0.0);
    k_gather_boxes<<<dim3((c->max_dof + 255) / 256, nsd), 256, 0, s>>>(smeta, md, scls, rin, rb);
    if (solve_f32(s, smeta, nsd, c->max_bt11, c->loc_solve4, c->loc_wide, 0, (const float*)(st + c->s_loc), scls, rb, zb, 1,
                  1 << 1, 1, scr, L.scr_stride, c->split11, (double*)(pb + L.sep), L.sep_q))
      return 1;
    k_scatter_boxes<<<dim3((c->max_dof + 255) / 256, nsd), 256, 0, s>>>(smeta, md, scls, zb, zout);
    k_coarse_restrict<<<nsd, 256, 0, s>>>(smeta, K, sV, rb, sroff, rc);
    if (tile_trsv(tiles, NT, NH, rc, ysc, xsc, s)) return 1;
    k_prolong<<<dim3((c->max_dof + 255) / 256, nsd), 256, 0, s>>>(smeta, md, K, sV, zero, xsc, sroff, zout, nullptr);
    return hipGetLastError() == hipSuccess ? 0 : 1;
  };
  CHIPCHK(c, hipMemcpyAsync(x, u, nd * 8, hipMemcpyDeviceToDevice, s));
  gspmv(x, q);
  k_sub<<<gblk, 256, 0, s>>>(gcls, nd, b, q, r);
  if (precond(r, z)) return cfail(c, MSGFEM_EHIP, "preconditioner launch failed");
  k_pcg_p<<<gblk, 256, 0, s>>>(gcls, nd, nullptr, z, pp);
  dot(r, z, sc + 0);
  dot(b, b, sc + 6);
  dot(r, r, sc + 3);
  CLAUNCHCHK(c);
  double h[8];
  CHIPCHK(c, hipMemcpyAsync(h, sc, 8 * 8, hipMemcpyDeviceToHost, s));
  CHIPCHK(c, hipStreamSynchronize(s));
  const double nb2 = h[6] > 0 ? std::sqrt(h[6]) : 1.0;
  double rel = std::sqrt(h[3]) / nb2;
  int it = 0;
  while (rel > rtol && it < maxit) {
    gspmv(pp, q);
    dot(pp, q, sc + 1);
    k_pcg_alpha<<<1, 1, 0, s>>>(sc);
    k_pcg_xr<<<gblk, 256, 0, s>>>(gcls, nd, sc, pp, q, x, r);
    dot(r, r, sc + 3);
    if (precond(r, z)) return cfail(c, MSGFEM_EHIP, "preconditioner launch failed");
    dot(r, z, sc + 2);
    k_pcg_beta<<<1, 1, 0, s>>>(sc);
    k_pcg_p<<<gblk, 256, 0, s>>>(gcls, nd, sc, z, pp);
    CLAUNCHCHK(c);
    // one 8-byte read per iteration (an iteration moves tens of GB at this size)
    CHIPCHK(c, hipMemcpyAsync(h + 3, sc + 3, 8, hipMemcpyDeviceToHost, s));
    CHIPCHK(c, hipStreamSynchronize(s));
    rel = std::sqrt(h[3]) / nb2;
    ++it;
  }
  CHIPCHK(c, hipMemcpyAsync(u, x, nd * 8, hipMemcpyDeviceToDevice, s));
  if (rel > rtol) k_status_or<<<1, 32, 0, s>>>(status, 1, 1);
  CLAUNCHCHK(c);
  CHIPCHK(c, hipStreamSynchronize(s));
  *iters = it;
  *relres = rel;
  return MSGFEM_OK;
}

extern "C" int msgfem_coarse_energy(msgfem_coarse* c, void* pcg, const double* u_ref, const double* u, double* out,
                                    void* stream) {
  if (!c || !pcg || !u_ref || !u || !out) return cfail(c, MSGFEM_EARG, "null argument");
  if (!c->geneo) return cfail(c, MSGFEM_EARG, "msgfem_coarse_energy reads the workspace of msgfem_coarse_pcg");
  CHIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  char* pb = (char*)pcg;
  const CPcgLayout L = cpcg_layout(c);
  const int64_t ng = c->n_nodes_global, nd = 3 * ng;
  const BoxMeta* gmeta = (const BoxMeta*)(pb + L.meta);
  const uint8_t* gcls = (const uint8_t*)(pb + L.cls);
  double *e = (double*)(pb + L.z), *Ae = (double*)(pb + L.q), *part = (double*)(pb + L.part);
  const unsigned gblk = (unsigned)std::min<int64_t>((nd + 255) / 256, 4096);
  const int gb = (int)((ng + 255) / 256);
  k_sub<<<gblk, 256, 0, s>>>(gcls, nd, u_ref, u, e);
  k_spmm<false, 1><<<dim3((unsigned)gb), 256, 0, s>>>(gmeta, 1, gb, (const double*)(pb + L.stencil), gcls,
                                                      (const double*)(pb + L.mu), e, Ae, nullptr, 1, 1 << 1, 1.0, nullptr);
  k_dot_partial<<<1024, 256, 0, s>>>(e, Ae, gcls, nd, part);
  k_dot_final<<<1, 256, 0, s>>>(part, 1024, out);
  k_spmm<false, 1><<<dim3((unsigned)gb), 256, 0, s>>>(gmeta, 1, gb, (const double*)(pb + L.stencil), gcls,
                                                      (const double*)(pb + L.mu), u_ref, Ae, nullptr, 1, 1 << 1, 1.0,
                                                      nullptr);
  k_dot_partial<<<1024, 256, 0, s>>>(u_ref, Ae, gcls, nd, part);
  k_dot_final<<<1, 256, 0, s>>>(part, 1024, out + 1);
  CLAUNCHCHK(c);
  return MSGFEM_OK;
}

// ------------------------------------------------------------ warm start
// every box of the batch has the node grid of box 0 (and so its DoF count)
static bool same_boxes(const msgfem_plan* p) {
  const BoxMeta& a = p->meta[0];
  for (const BoxMeta& b : p->meta)
    if (b.mx != a.mx || b.my != a.my || b.mz != a.mz) return false;
  return true;
}

extern "C" int msgfem_warm_features(msgfem_plan* p, const void* ops, float* feat, void* stream) {
  if (!p || !ops || !feat) return fail(p, MSGFEM_EARG, "null argument");
  if (!same_boxes(p)) return fail(p, MSGFEM_EARG, "warm start needs boxes of one node grid");
  if (set_device(p)) return MSGFEM_EHIP;
  OpsView v = ops_view(p, ops);
  const BoxMeta& a = p->meta[0];
  const int ne = (a.mx - 1) * (a.my - 1) * (a.mz - 1);
  k_warm_features<<<dim3((ne + 255) / 256, (unsigned)p->meta.size()), 256, 0, (hipStream_t)stream>>>(
      v.meta, mesh_dev(p), feat);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_warm_basis(msgfem_plan* p, const void* ops, const double* evecs, int32_t ng, double* G,
                                 void* stream) {
  if (!p || !ops || !evecs || !G) return fail(p, MSGFEM_EARG, "null argument");
  const BoxMeta& a = p->meta[0];
  if (ng < 1 || ng > a.n_ev) return fail(p, MSGFEM_EARG, "ng must be in [1, n_ev of box 0 = %d]", a.n_ev);
  if (set_device(p)) return MSGFEM_EHIP;
  OpsView v = ops_view(p, ops);
  k_warm_basis<<<1, 1024, 0, (hipStream_t)stream>>>(v.meta, v.cls, evecs + a.evec_off, a.n_ev, ng, G);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_warm_labels(msgfem_plan* p, const void* ops, const double* evecs, const double* G,
                                  int32_t n_dof_g, int32_t ng, int32_t ne, float* P, void* stream) {
  if (!p || !ops || !evecs || !G || !P) return fail(p, MSGFEM_EARG, "null argument");
  if (!same_boxes(p) || p->meta[0].n_dof != n_dof_g)
    return fail(p, MSGFEM_EARG, "every box must have the %d DoFs of the basis", n_dof_g);
  for (const BoxMeta& b : p->meta)
    if (ne < 1 || ne > b.n_ev) return fail(p, MSGFEM_EARG, "ne must be in [1, n_ev]");
  if (ng < ne || (int64_t)ng * ne * 8 > 64 * 1024) return fail(p, MSGFEM_EARG, "need ne <= ng, ng*ne <= 8192");
  if (set_device(p)) return MSGFEM_EHIP;
  OpsView v = ops_view(p, ops);
  k_warm_labels<<<(unsigned)p->meta.size(), 256, (size_t)ng * ne * 8, (hipStream_t)stream>>>(v.meta, v.cls, evecs,
                                                                                            G, ng, ne, P);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}

extern "C" int msgfem_warm_start(msgfem_plan* p, const void* ops, const float* coef, const double* G,
                                 int32_t n_dof_g, int32_t ng, int32_t ne, uint64_t seed, double* x0,
                                 void* stream) {
  if (!p || !ops || !coef || !G || !x0) return fail(p, MSGFEM_EARG, "null argument");
  if (!same_boxes(p) || p->meta[0].n_dof != n_dof_g)
    return fail(p, MSGFEM_EARG, "every box must have the %d DoFs of the basis", n_dof_g);
  if (ng < 1 || ne < 0 || ne > p->k) return fail(p, MSGFEM_EARG, "need ng >= 1 and 0 <= ne <= block %d", p->k);
  if ((int64_t)ng * ne > 12288) return fail(p, MSGFEM_EARG, "ng x ne = %d exceeds 12288", ng * ne);
  if (set_device(p)) return MSGFEM_EHIP;
  OpsView v = ops_view(p, ops);
  const size_t lds = ((size_t)ng * ne + ne) * 4;
  k_warm_start<<<dim3((unsigned)((n_dof_g + 255) / 256), (unsigned)p->meta.size()), 256, lds,
                 (hipStream_t)stream>>>(v.meta, v.cls, coef, G, ng, ne, p->k, seed, x0);
  LAUNCHCHK(p);
  return MSGFEM_OK;
}
