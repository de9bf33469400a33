// Internal data structures of libpfrac (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pf.h"

namespace pf {

constexpr int kBlock = 256;          // threads per workgroup of every tile kernel (4 wave64s)
constexpr int kMaxTileNodes = 2048;  // owned nodes per tile, upper limit
constexpr int kWaves = kBlock / 64;

// One tile: a contiguous range of owned nodes plus the halo needed to
// evaluate every element that touches them.  The tile's element list is in
// ascending internal element id; the owned elements carry consecutive ids, so
// they form one run of it, and every owned node's corner list (ascending
// element id) is ascending in the local element index too.
struct TileRec {
  int32_t node_begin;      // first owned node (internal id)
  int32_t n_own;           // owned nodes
  int32_t halo_begin;      // offset into halo_idx
  int32_t n_halo;          // halo nodes (local ids n_own .. n_own+n_halo-1)
  int32_t telem_begin;     // offset into the tile-element arrays
  int32_t n_telem;         // elements evaluated by this tile (owned + halo)
  int32_t n_own_elem;      // owned elements, local indices own_elem_lo .. own_elem_lo + n_own_elem - 1
  int32_t own_elem_begin;  // internal id of the first owned element
  int32_t inst;            // instance
  int32_t lds_bytes;       // dynamic LDS this tile needs (explicit kernel, FP64 upper bound)
  int32_t corner_begin;    // first entry of the owned nodes' corner lists (lcorner index)
  int32_t n_corner;        // entries in the owned nodes' corner lists
  int32_t own_elem_lo;     // local index of the first owned element
};

// Per-instance constants for the kernels, in the arithmetic type T.
template <typename T>
struct InstP {
  // explicit step
  T dt, half_dt, half_dt2, inv_rho;
  T lam, mu, Kc2, coef, gamma, eta;
  // damage system scaled by s = l0/Gc:  A~ = kap K + sum (c0 + cH H_e) M^e,
  // b~_i = sum (b0 + bH H_e) A_e/3
  T kap, c0, cH, b0, bH;
  // d(scaled operator)/dGc terms for the adjoint, scaled by 1/Gc (see adjoint.hip)
  T gK, gM, gW;            // dL/dGc += -lam~'(gK K d + gM M d + gW w)
  T tol;
  // fracture energy (per unit thickness): efr * (d'Md + l0sq d'Kd) for AT2
  // (efr = Gc/(2 l0)), efr * (int d + l0sq d'Kd) for AT1 (efr = 3 Gc/(8 l0))
  T efr, l0sq;
  int32_t model, bounds, split, pad;
  double dtd;              // dt in FP64 (advances the state time)
};

// Ramped loads registered by pf_set_loading: ramp times of one instance.
struct LoadP {
  double t_f;              // traction ramp time (<= 0: S = 1 for t > 0)
  double t_v;              // velocity ramp time (<= 0: R = 1)
};

// Device view of the registered loads; par is null when none are registered.
struct LoadDev {
  const void* F;           // [2][N] full-load nodal force (mesh dtype) or null
  const void* vfull;       // [2][N] prescribed velocity at full ramp (mesh dtype) or null
  const LoadP* par;        // [n_inst]
};

// CG control block of one instance, in device memory.  Fields are read by
// every block at kernel start and written only by the instance's last block.
struct Ctl {
  int32_t mode;       // MODE_*
  int32_t setup;      // 1 on the first restart of a solve (assemble b and the diagonal)
  int32_t release;    // the pending restart may release nodes held at the bound
  int32_t hit;        // the current step is cut by a bound
  int32_t iters, restarts, flags, nact;
  int32_t pbuf;       // which half of the vector pairs (x, r, A z, A p) is current
  int32_t ntiles;     // tiles of this instance
  int32_t tile0;      // first tile of this instance
  int32_t flavor;     // 0 active-set updates between CG runs, 1 monotone projected CG (fallback)
  int32_t nnodes;     // nodes of this instance
  int32_t inner;      // CG iterations since the last restart or check
  int32_t wbuf;       // which half of the held-set pair is current
  int32_t outer;      // active-set updates so far
  int32_t cbase;      // first arrival counter of this instance (counters of 32-tile groups, then the top one)
  int32_t ngroup;     // 32-tile groups of this instance
  double rz, alpha, beta, amax, resid, pq;
  double ref;         // scale of the stopping test (1 for the damage QP, max |b_i|/A_ii for linear solves)
  double lmax;        // upper bound of the spectrum of D^-1 A (set-up pass; Chebyshev preconditioner)
};

enum { MODE_RESTART = 0, MODE_ITER = 1, MODE_DONE = 2, MODE_CHECK = 3, MODE_FIRST = 4 };

// Arrival counting of the damage passes: tiles of an instance count in groups
// of kArriveGroup, the last of each group counts at the instance's top counter.
// Counters sit kArriveStride uint32 apart (one 128-byte line each).
constexpr int kArriveGroup = 32;
constexpr int kArriveStride = 32;

// Device view of a mesh handle.
struct DevMesh {
  const TileRec* tiles;
  const int32_t* halo_idx;      // [sum n_halo] internal node ids
  const uint16_t* lc0;          // [n_te] local node index of corner 0/1/2
  const uint16_t* lc1;
  const uint16_t* lc2;
  const int32_t* te_gid;        // [n_te] internal element id of each tile element
  const void* geo;              // [7][n_te] gx0 gy0 gx1 gy1 gx2 gy2 area (mesh dtype)
  const void* kw;               // [3][n_te] element stiffness off-diagonals K01 K02 K12 (mesh dtype)
  const int32_t* lrow;          // [N+1] corner list range of each owned node
  const uint16_t* lcorner;      // [sum] tile-local corner id 3*e+k, ascending element id
  const void* inv_w;            // [N] 1 / sum_{e ni i} A_e/3 (mesh dtype)
  const void* wlump;            // [N] sum_{e ni i} A_e/3 (mesh dtype)
  const uint8_t* fixed;         // [N] bit0 x prescribed, bit1 y prescribed
  const void* gcs;              // [n_te] toughness factor phi_e = Gc_e / Gc of each tile element
                                // (mesh dtype), or null for a uniform Gc
  int32_t n_nodes, n_elems, n_tiles, n_te;
};

// Device workspaces of the damage solve and of the adjoint.
struct DevWork {
  void* b; void* dinv;               // [n_nodes] CG load vector and Jacobi diagonal inverse
  void* r0; void* r1;                // [n_nodes] residual pair
  void* w0; void* w1;                // [n_nodes] A z pair
  void* s0; void* s1;                // [n_nodes] A p pair
  void* p;                           // [n_nodes] search direction
  void* xw0; void* xw1;              // [n_nodes] iterate pair of the damage solve
  void* zb;                          // [n_nodes] z = M r of the current iteration (polynomial preconditioner)
  void* y0; void* y1;                // [n_nodes] Chebyshev iterate pair (polynomial preconditioner)
  void* dv;                          // [n_nodes] Chebyshev update direction (polynomial preconditioner)
  uint8_t* wset;                     // [2][n_nodes] held-set pair
  void* lam;                         // [n_nodes] adjoint multiplier (warm start of the next adjoint solve)
  void* lam_prev;                    // [n_nodes] the multiplier of the call before (linear extrapolation)
  void* hbar;                        // [n_elems] adjoint of H_{n+1} (adjoint step scratch)
  void* mte;                         // [n_te] per-solve mass coefficient (c0 + cH H_e) A_e / 12 of each tile element
  double* part;                      // [n_tiles][8] block partials
  uint32_t* arrive;                  // arrival counters of the damage passes, kArriveStride apart:
                                     // per instance one per 32-tile group, then one for the groups
  Ctl* ctl;                          // [n_inst]
  void* instp;                       // [n_inst] InstP<T>
  int* bounds;                       // [n_inst] pf_params_t.bounds of each instance
};

struct Timer {
  std::vector<hipEvent_t> ev;        // pairs
  size_t used = 0;
  double ms = 0.0;
  int64_t launches = 0;
};

}  // namespace pf

struct pf_mesh_s {
  pf_dtype_t dtype;
  int32_t n_inst = 0, n_nodes = 0, n_elems = 0, n_tiles = 0, n_te = 0;
  int32_t max_tile_nodes = 0, max_tile_elems = 0, max_own = 0, max_lds_explicit = 0, max_lds_damage = 0;
  int32_t max_corner = 0;
  int32_t max_inst_tiles = 0;        // tiles of the largest instance
  size_t adj_lds_damage = 0;         // LDS of the adjoint kernels (set by the first backward step)
  size_t adj_lds_explicit = 0;
  int32_t adj_chunks = 0;            // element chunks of the explicit step's adjoint (0: not yet chosen)
  int64_t adj_calls = 0;             // pf_step_backward calls on this handle
  int32_t explicit_block = 256;      // workgroup size of the explicit-step kernel (256 or 512)
  int32_t max_lds_explicit2 = 0;     // LDS of the explicit step with its elements in two chunks
  int32_t explicit_chunks = 0;       // 1, 2, or 0 = automatic
  int32_t max_lds_damage2 = 0;       // LDS of the damage passes with their elements in two chunks
  int32_t damage_chunks = 0;         // as requested: 1, 2, or 0 = automatic
  int32_t dmg_nch = 0;               // element chunks of the damage passes (0: not yet chosen)
  int32_t lds_per_cu = 160 * 1024;   // device limits that set how many workgroups share a CU
  int32_t threads_per_cu = 2048;
  int32_t split = -1;
  std::vector<pf_instance_info_t> info;
  std::vector<int32_t> node_perm, elem_perm;
  std::vector<pf::TileRec> tiles_h;
  pf::DevMesh dm{};
  pf::DevWork dw{};
  std::vector<void*> allocs;         // every device allocation, freed at destroy
  size_t device_bytes = 0;
  // host mirror of the current per-instance parameters (bytes of InstP<T>[n_inst])
  // and of their bounds modes; sized at create, valid once uploaded
  std::vector<unsigned char> instp_host;
  std::vector<int32_t> bounds_host;
  bool params_valid = false;
  int32_t device = 0;                // HIP device the handle was created on
  std::vector<double> dt_cache;      // dt of the last explicit step (the damage solve reuses it)
  int32_t last_rounds[2] = {0, 0};   // CG rounds the last solve of each kind needed (sets the first poll)
  bool qp_started = false;           // a damage solve has been enqueued (resume is allowed)
  std::vector<unsigned char> last_qp_args;   // kernel arguments of the last damage solve's passes
  int32_t last_qp_cheb = 0;                  // its polynomial degree (0: Jacobi)
  pf::Ctl* ctl_pinned = nullptr;     // pinned host copy of the control blocks
  hipEvent_t poll_ev = nullptr;      // marks the copy of the control blocks (convergence polls)
  bool timing = false;
  pf::Timer timers[5];
  void* gcs_buf = nullptr;           // device storage of dm.gcs (allocated by the first pf_set_gc_field)
  double* dgc_field = nullptr;       // caller's per-element dL/dGc_e accumulator, or null
  void* load_buf = nullptr;          // device storage of the loads (allocated by the first pf_set_loading)
  pf::LoadDev ld{};                  // the registered loads (ld.par null: none)
};

namespace pf {

void set_error(const std::string& s);
pf_status_t fail(pf_status_t st, const std::string& s);
pf_status_t hip_fail(hipError_t e, const char* what);

#define PF_HIP(call)                                          \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::pf::hip_fail(e_, #call);   \
  } while (0)

// Fill the per-instance constants for dtype T; uploads them if they changed.
pf_status_t upload_params(pf_mesh_s* m, const pf_params_t* p, const double* dt, hipStream_t s);

// Kernel timing around launches.
void timer_begin(pf_mesh_s* m, int family, hipStream_t s);
void timer_end(pf_mesh_s* m, int family, hipStream_t s);

inline size_t elem_size(pf_dtype_t t) { return t == PF_F64 ? 8 : 4; }

pf_status_t check_params(const pf_mesh_s* m, const pf_params_t* p, const double* dt, bool need_dt);

// Matrix-free CG on the damage operator (damage.hip).  kind 0: the bound-
// constrained damage update (b assembled from H, lower bound lb, result in x).
// kind 1: the linear system A_FF x_F = b_F on the fixed free set F = {W == 0}
// (b, W and the starting x prepared by the caller in the workspaces; the
// stopping test is relative to max |b_i|/A_ii).
enum { CG_QP = 0, CG_LINEAR = 1 };
pf_status_t damage_cg(pf_mesh_s* m, int kind, const void* H, const void* lb, void* x, const uint8_t* guess,
                      uint8_t* active_out, const pf_cg_opts_t* o, pf_cg_stats_t* stats, hipStream_t s);
pf_status_t check_state(const pf_state_t* s, bool need_d, bool need_H, const char* name);
// Resolve, once per device (that device current), the device address of the
// static partials array of pf_energies_static (energy.hip).
pf_status_t energy_scratch_setup(int device);
// Choose the element chunks of the damage passes for this handle (damage.hip).
void damage_plan(pf_mesh_s* m);
bool states_share(const pf_state_t* a, const pf_state_t* b);

}  // namespace pf
