// Mesh handle: validation, P1 geometry (eq. grad_phi, lumped mass), tile plan,
// device upload, per-instance parameters, error reporting and kernel timers.
#include <algorithm>
#include <iterator>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "pf_internal.hpp"

namespace pf {

static thread_local std::string g_err;

void set_error(const std::string& s) { g_err = s; }

pf_status_t fail(pf_status_t st, const std::string& s) {
  g_err = s;
  return st;
}

pf_status_t hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return PF_ERR_HIP;
}

namespace {

struct Geo {
  double g[6];   // gx0 gy0 gx1 gy1 gx2 gy2
  double area;
};

// Recursive coordinate bisection: split [lo, hi) of ids along the longer
// side of its bounding box until a part holds at most maxn nodes.  The split
// point is proportional to the number of leaves on each side so that leaves
// come out nearly equal.  Ties are broken by node id (deterministic).
void rcb(std::vector<int32_t>& ids, size_t lo, size_t hi, const double* xy, size_t maxn,
         std::vector<std::pair<size_t, size_t>>& leaves) {
  size_t n = hi - lo;
  if (n <= maxn) {
    leaves.emplace_back(lo, hi);
    return;
  }
  double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
  for (size_t i = lo; i < hi; ++i)
    for (int a = 0; a < 2; ++a) {
      mn[a] = std::min(mn[a], xy[2 * ids[i] + a]);
      mx[a] = std::max(mx[a], xy[2 * ids[i] + a]);
    }
  int ax = (mx[0] - mn[0] >= mx[1] - mn[1]) ? 0 : 1;
  size_t nl = (n + maxn - 1) / maxn;
  size_t mid = lo + (n * (nl / 2)) / nl;
  std::nth_element(ids.begin() + lo, ids.begin() + mid, ids.begin() + hi, [&](int32_t a, int32_t b) {
    double ca = xy[2 * a + ax], cb = xy[2 * b + ax];
    return ca < cb || (ca == cb && a < b);
  });
  rcb(ids, lo, mid, xy, maxn, leaves);
  rcb(ids, mid, hi, xy, maxn, leaves);
}

template <typename T>
void to_dtype(const std::vector<double>& src, std::vector<unsigned char>& dst) {
  dst.resize(src.size() * sizeof(T));
  T* p = reinterpret_cast<T*>(dst.data());
  for (size_t i = 0; i < src.size(); ++i) p[i] = static_cast<T>(src[i]);
}

}  // namespace

pf_status_t check_params(const pf_mesh_s* m, const pf_params_t* p, const double* dt, bool need_dt) {
  if (!p) return fail(PF_ERR_ARG, "params is NULL");
  if (need_dt && !dt) return fail(PF_ERR_ARG, "dt is NULL");
  for (int k = 0; k < m->n_inst; ++k) {
    const pf_params_t& q = p[k];
    auto bad = [&](const char* what) { return fail(PF_ERR_ARG, "instance " + std::to_string(k) + ": " + what); };
    if (!(q.E > 0) || !std::isfinite(q.E)) return bad("E must be > 0");
    if (!(q.nu >= 0 && q.nu < 0.5)) return bad("nu must be in [0, 0.5)");
    if (!(q.rho > 0) || !std::isfinite(q.rho)) return bad("rho must be > 0");
    if (!(q.Gc > 0) || !std::isfinite(q.Gc)) return bad("Gc must be > 0");
    if (!(q.l0 > 0) || !std::isfinite(q.l0)) return bad("l0 must be > 0");
    if (!(q.eta >= 0) || !std::isfinite(q.eta)) return bad("eta must be >= 0");
    if (!(q.gamma_star >= 0) || !std::isfinite(q.gamma_star)) return bad("gamma_star must be >= 0");
    if (q.model != PF_AT1 && q.model != PF_AT2) return bad("model must be 1 (AT1) or 2 (AT2)");
    if (q.split < 0 || q.split > 3) return bad("split must be 0..3");
    if (q.plane != PF_PLANE_STRAIN && q.plane != PF_PLANE_STRESS) return bad("plane must be 0 or 1");
    if (q.bounds != PF_BOUNDS_PROJECTED && q.bounds != PF_BOUNDS_POSTCLAMP) return bad("bounds must be 0 or 1");
    if (q.bounds == PF_BOUNDS_POSTCLAMP && q.model != PF_AT2) return bad("post-clamp bounds need AT2");
    if (q.split != p[0].split) return fail(PF_ERR_UNSUPPORTED, "all instances of a handle must use one split");
    if (need_dt && (!(dt[k] > 0) || !std::isfinite(dt[k]))) return bad("dt must be > 0");
  }
  return PF_OK;
}

template <typename T>
static void fill_instp(const pf_params_t& q, double dt, InstP<T>& o) {
  const double E = q.E, nu = q.nu;
  const double mu = E / (2.0 * (1.0 + nu));
  const double lam_pe = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double lam_ps = E * nu / (1.0 - nu * nu);
  const double K = E / (3.0 * (1.0 - 2.0 * nu));
  const double s = (q.plane == PF_PLANE_STRESS) ? -nu / (1.0 - nu) : 0.0;
  const double c = 1.0 + s;
  const double lam = (q.plane == PF_PLANE_STRESS) ? lam_ps : lam_pe;
  std::memset(&o, 0, sizeof(o));
  o.dt = T(dt);
  o.dtd = dt;
  o.half_dt = T(0.5 * dt);
  o.half_dt2 = T(0.5 * dt * dt);
  o.inv_rho = T(1.0 / q.rho);
  o.lam = T(lam);
  o.mu = T(mu);
  o.Kc2 = T(K * c * c);
  o.coef = T(s * s - c * c / 3.0);
  o.gamma = T(q.split == PF_SPLIT_STARCONVEX ? q.gamma_star : 0.0);
  o.eta = T(q.eta);
  o.efr = T(q.model == PF_AT2 ? q.Gc / (2.0 * q.l0) : 3.0 * q.Gc / (8.0 * q.l0));
  o.l0sq = T(q.l0 * q.l0);
  const double sc = q.l0 / q.Gc;   // the damage system is scaled by l0/Gc
  if (q.model == PF_AT2) {
    o.kap = T(q.l0 * q.l0);
    o.c0 = T(1.0);
    o.b0 = T(0.0);
    o.gK = T(q.l0 * q.l0 / q.Gc);
    o.gM = T(1.0 / q.Gc);
    o.gW = T(0.0);
  } else {
    o.kap = T(0.75 * q.l0 * q.l0);
    o.c0 = T(0.0);
    o.b0 = T(-0.375);
    o.gK = T(0.75 * q.l0 * q.l0 / q.Gc);
    o.gM = T(0.0);
    o.gW = T(0.375 / q.Gc);
  }
  o.cH = T(2.0 * sc);
  o.bH = T(2.0 * sc);
  o.model = q.model;
  o.bounds = q.bounds;
  o.split = q.split;
}

pf_status_t upload_params(pf_mesh_s* m, const pf_params_t* p, const double* dt, hipStream_t s) {
  // No allocation here: the host mirror and the bounds array are sized by
  // pf_mesh_create, and each instance's constants are formed on the stack.
  const size_t sz = (m->dtype == PF_F64) ? sizeof(InstP<double>) : sizeof(InstP<float>);
  if (!dt && !m->dt_cache.empty()) dt = m->dt_cache.data();
  bool changed = !m->params_valid;
  for (int k = 0; k < m->n_inst; ++k) {
    const double d = dt ? dt[k] : 0.0;
    union {
      InstP<double> f64;
      InstP<float> f32;
    } q;
    if (m->dtype == PF_F64)
      fill_instp<double>(p[k], d, q.f64);
    else
      fill_instp<float>(p[k], d, q.f32);
    unsigned char* dst = m->instp_host.data() + sz * size_t(k);
    if (std::memcmp(dst, &q, sz) != 0) {
      std::memcpy(dst, &q, sz);
      changed = true;
    }
    if (m->bounds_host[k] != p[k].bounds) {
      m->bounds_host[k] = p[k].bounds;
      changed = true;
    }
  }
  if (changed) {
    // Parameters change rarely (a new Gc or dt); a blocking copy keeps the
    // host buffer's lifetime trivial.
    PF_HIP(hipStreamSynchronize(s));
    PF_HIP(hipMemcpy(m->dw.instp, m->instp_host.data(), sz * size_t(m->n_inst), hipMemcpyHostToDevice));
    PF_HIP(hipMemcpy(m->dw.bounds, m->bounds_host.data(), sizeof(int) * size_t(m->n_inst), hipMemcpyHostToDevice));
    m->params_valid = true;
  }
  return PF_OK;
}

void timer_begin(pf_mesh_s* m, int family, hipStream_t s) {
  if (!m->timing) return;
  Timer& t = m->timers[family];
  if (2 * t.used + 2 > t.ev.size()) {
    // pool exhausted: fold the recorded pairs into the running total
    if (!t.ev.empty()) {
      (void)hipEventSynchronize(t.ev[2 * t.used - 1]);
      for (size_t k = 0; k < t.used; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]);
        t.ms += ms;
      }
      t.used = 0;
    }
    if (t.ev.empty()) {
      t.ev.resize(2 * 4096);
      // no system-scope fence: the events only time kernels on this device
      for (auto& e : t.ev) (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    }
  }
  (void)hipEventRecord(t.ev[2 * t.used], s);
}

void timer_end(pf_mesh_s* m, int family, hipStream_t s) {
  if (!m->timing) return;
  Timer& t = m->timers[family];
  (void)hipEventRecord(t.ev[2 * t.used + 1], s);
  ++t.used;
  ++t.launches;
}

}  // namespace pf

using namespace pf;

extern "C" const char* pf_last_error(void) { return pf::g_err.c_str(); }

extern "C" const char* pf_version(void) { return "libpfrac 0.1 (gfx950)"; }

template <typename Tp>
static pf_status_t dev_upload(pf_mesh_s* m, const std::vector<Tp>& h, void** out) {
  size_t bytes = std::max<size_t>(h.size() * sizeof(Tp), 16);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(PF_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  m->allocs.push_back(p);
  m->device_bytes += bytes;
  if (!h.empty()) PF_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(Tp), hipMemcpyHostToDevice));
  *out = p;
  return PF_OK;
}

static pf_status_t dev_alloc(pf_mesh_s* m, size_t bytes, void** out) {
  bytes = std::max<size_t>(bytes, 16);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(PF_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  m->allocs.push_back(p);
  m->device_bytes += bytes;
  PF_HIP(hipMemset(p, 0, bytes));
  *out = p;
  return PF_OK;
}

static void free_all(pf_mesh_s* m) {
  for (void* p : m->allocs) (void)hipFree(p);
  m->allocs.clear();
  if (m->ctl_pinned) (void)hipHostFree(m->ctl_pinned);
  m->ctl_pinned = nullptr;
  if (m->poll_ev) (void)hipEventDestroy(m->poll_ev);
  m->poll_ev = nullptr;
  for (auto& t : m->timers)
    for (auto& e : t.ev) (void)hipEventDestroy(e);
}

extern "C" pf_status_t pf_mesh_create(const pf_mesh_desc_t* inst, int32_t n_instances, pf_dtype_t dtype,
                                      const pf_tile_opts_t* tile, pf_stream_t stream, pf_mesh_t* out) {
  if (!out) return fail(PF_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!inst || n_instances < 1) return fail(PF_ERR_ARG, "need at least one instance");
  if (dtype != PF_F32 && dtype != PF_F64) return fail(PF_ERR_ARG, "dtype must be PF_F32 or PF_F64");
  int tile_nodes = (tile && tile->tile_nodes > 0) ? tile->tile_nodes : (dtype == PF_F64 ? 256 : 512);
  if (tile_nodes < 64 || tile_nodes > kMaxTileNodes) return fail(PF_ERR_ARG, "tile_nodes must be in [64, 2048]");
  const int explicit_block = (tile && tile->explicit_block > 0) ? tile->explicit_block : kBlock;
  if (explicit_block != 256 && explicit_block != 512) return fail(PF_ERR_ARG, "explicit_block must be 256 or 512");
  const int explicit_chunks = tile ? tile->explicit_chunks : 0;
  if (explicit_chunks < 0 || explicit_chunks > 2) return fail(PF_ERR_ARG, "explicit_chunks must be 0, 1 or 2");
  const int damage_chunks = tile ? tile->damage_chunks : 0;
  if (damage_chunks < 0 || damage_chunks > 2) return fail(PF_ERR_ARG, "damage_chunks must be 0, 1 or 2");

  // ---- validate and count -------------------------------------------------
  int64_t n_tot = 0, e_tot = 0;
  for (int k = 0; k < n_instances; ++k) {
    const pf_mesh_desc_t& d = inst[k];
    if (d.n_nodes < 3 || d.n_elems < 1 || !d.xy || !d.tri)
      return fail(PF_ERR_ARG, "instance " + std::to_string(k) + ": empty mesh or NULL array");
    n_tot += d.n_nodes;
    e_tot += d.n_elems;
  }
  if (n_tot >= (int64_t(1) << 31) - 1 || 3 * e_tot >= (int64_t(1) << 31) - 1)
    return fail(PF_ERR_ARG, "mesh too large for 32-bit indices");

  pf_mesh_s* m = new (std::nothrow) pf_mesh_s();
  if (!m) return fail(PF_ERR_NOMEM, "host allocation failed");
  m->dtype = dtype;
  m->explicit_block = explicit_block;
  m->explicit_chunks = explicit_chunks;
  m->damage_chunks = damage_chunks;
  m->n_inst = n_instances;
  m->n_nodes = int32_t(n_tot);
  m->n_elems = int32_t(e_tot);
  m->info.resize(n_instances);
  m->node_perm.resize(n_tot);
  m->elem_perm.resize(e_tot);

  std::vector<double> geo_te[7];                   // tile-element geometry, FP64
  std::vector<uint16_t> lc[3];
  std::vector<int32_t> te_gid, halo_idx, lrow(n_tot + 1, 0);
  std::vector<uint16_t> lcorner;
  std::vector<double> inv_w(n_tot), wl(n_tot);
  std::vector<uint8_t> fixed(n_tot, 0);
  lcorner.reserve(size_t(e_tot) * 3);

  int32_t node_off = 0, elem_off = 0;
  for (int k = 0; k < n_instances; ++k) {
    const pf_mesh_desc_t& d = inst[k];
    const int32_t n = d.n_nodes, ne = d.n_elems;
    auto mesh_err = [&](const std::string& s) {
      delete m;
      return fail(PF_ERR_MESH, "instance " + std::to_string(k) + ": " + s);
    };
    // orientation and geometry (eq. grad_phi), FP64
    std::vector<int32_t> tri(size_t(ne) * 3);
    std::vector<Geo> geo(ne);
    std::vector<int32_t> deg(n, 0);
    double hmin = INFINITY, area_sum = 0.0;
    for (int32_t i = 0; i < 2 * n; ++i)
      if (!std::isfinite(d.xy[i])) return mesh_err("non-finite coordinate");
    for (int32_t e = 0; e < ne; ++e) {
      int32_t a = d.tri[3 * e], b = d.tri[3 * e + 1], c = d.tri[3 * e + 2];
      if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n)
        return mesh_err("element " + std::to_string(e) + " has a node index out of range");
      if (a == b || b == c || a == c) return mesh_err("element " + std::to_string(e) + " repeats a node");
      double x1 = d.xy[2 * a], y1 = d.xy[2 * a + 1];
      double x2 = d.xy[2 * b], y2 = d.xy[2 * b + 1];
      double x3 = d.xy[2 * c], y3 = d.xy[2 * c + 1];
      double two_a = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
      if (!(two_a != 0.0) || !std::isfinite(two_a)) return mesh_err("element " + std::to_string(e) + " has zero area");
      if (two_a < 0) {
        std::swap(b, c);
        std::swap(x2, x3);
        std::swap(y2, y3);
        two_a = -two_a;
      }
      tri[3 * e] = a;
      tri[3 * e + 1] = b;
      tri[3 * e + 2] = c;
      Geo& g = geo[e];
      g.g[0] = (y2 - y3) / two_a;
      g.g[1] = (x3 - x2) / two_a;
      g.g[2] = (y3 - y1) / two_a;
      g.g[3] = (x1 - x3) / two_a;
      g.g[4] = (y1 - y2) / two_a;
      g.g[5] = (x2 - x1) / two_a;
      g.area = 0.5 * two_a;
      area_sum += g.area;
      double per = std::hypot(x2 - x1, y2 - y1) + std::hypot(x3 - x2, y3 - y2) + std::hypot(x1 - x3, y1 - y3);
      hmin = std::min(hmin, 4.0 * g.area / per);
      deg[a]++, deg[b]++, deg[c]++;
    }
    for (int32_t i = 0; i < n; ++i)
      if (deg[i] == 0) return mesh_err("node " + std::to_string(i) + " belongs to no element");
    // node -> element adjacency (user ids)
    std::vector<int32_t> adj_ptr(n + 1, 0), adj(size_t(ne) * 3);
    for (int32_t i = 0; i < n; ++i) adj_ptr[i + 1] = adj_ptr[i] + deg[i];
    {
      std::vector<int32_t> fill(adj_ptr.begin(), adj_ptr.end() - 1);
      for (int32_t e = 0; e < ne; ++e)
        for (int q = 0; q < 3; ++q) adj[fill[tri[3 * e + q]]++] = e;
    }
    // tiles by recursive coordinate bisection
    std::vector<int32_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0);
    std::vector<std::pair<size_t, size_t>> leaves;
    rcb(ids, 0, n, d.xy, size_t(tile_nodes), leaves);
    std::vector<int32_t> node_int(n), node_tile(n);   // user -> internal (instance-local), tile (global)
    int32_t tile0 = int32_t(m->tiles_h.size());
    {
      int32_t pos = 0;
      for (size_t t = 0; t < leaves.size(); ++t) {
        std::sort(ids.begin() + leaves[t].first, ids.begin() + leaves[t].second);
        for (size_t i = leaves[t].first; i < leaves[t].second; ++i) {
          node_int[ids[i]] = pos++;
          node_tile[ids[i]] = tile0 + int32_t(t);
        }
      }
    }
    for (int32_t i = 0; i < n; ++i) {
      m->node_perm[node_off + node_int[i]] = i;
      double wsum = 0.0;
      for (int32_t j = adj_ptr[i]; j < adj_ptr[i + 1]; ++j) wsum += geo[adj[j]].area / 3.0;
      wl[node_off + node_int[i]] = wsum;
      inv_w[node_off + node_int[i]] = 1.0 / wsum;
      if (d.fixed) fixed[node_off + node_int[i]] = uint8_t((d.fixed[2 * i] ? 1 : 0) | (d.fixed[2 * i + 1] ? 2 : 0));
    }
    // element owner = tile of the element's smallest internal node id
    std::vector<int32_t> emin(ne), eorder(ne), elem_int(ne);
    for (int32_t e = 0; e < ne; ++e)
      emin[e] = std::min({node_int[tri[3 * e]], node_int[tri[3 * e + 1]], node_int[tri[3 * e + 2]]});
    std::iota(eorder.begin(), eorder.end(), 0);
    std::stable_sort(eorder.begin(), eorder.end(), [&](int32_t a, int32_t b) { return emin[a] < emin[b]; });
    for (int32_t j = 0; j < ne; ++j) {
      elem_int[eorder[j]] = j;
      m->elem_perm[elem_off + j] = eorder[j];
    }
    auto owner = [&](int32_t e) { return node_tile[m->node_perm[node_off + emin[e]]]; };
    // per tile lists
    const int32_t nt = int32_t(leaves.size());
    int32_t own_elem_cursor = 0;
    int32_t node_cursor = 0;
    for (int32_t t = 0; t < nt; ++t) {
      const int32_t gt = tile0 + t;
      TileRec rec{};
      rec.inst = k;
      rec.node_begin = node_off + node_cursor;
      rec.n_own = int32_t(leaves[t].second - leaves[t].first);
      // owned nodes in internal order (user ids)
      std::vector<int32_t> own_user(rec.n_own);
      for (int32_t i = 0; i < rec.n_own; ++i) own_user[i] = m->node_perm[node_off + node_cursor + i];
      // elements touching an owned node
      std::vector<int32_t> owned_e, halo_e;
      for (int32_t u : own_user)
        for (int32_t j = adj_ptr[u]; j < adj_ptr[u + 1]; ++j) {
          int32_t e = adj[j];
          (owner(e) == gt ? owned_e : halo_e).push_back(e);
        }
      auto by_int = [&](int32_t a, int32_t b) { return elem_int[a] < elem_int[b]; };
      std::sort(owned_e.begin(), owned_e.end(), by_int);
      owned_e.erase(std::unique(owned_e.begin(), owned_e.end()), owned_e.end());
      std::sort(halo_e.begin(), halo_e.end(), by_int);
      halo_e.erase(std::unique(halo_e.begin(), halo_e.end()), halo_e.end());
      rec.n_own_elem = int32_t(owned_e.size());
      rec.own_elem_begin = elem_off + own_elem_cursor;
      for (int32_t j = 0; j < rec.n_own_elem; ++j)
        if (elem_int[owned_e[j]] != own_elem_cursor + j) {
          delete m;
          return fail(PF_ERR_MESH, "internal: owned elements are not contiguous");
        }
      own_elem_cursor += rec.n_own_elem;
      // tile elements in ascending internal id: halo elements of earlier
      // tiles, the owned run, then halo elements of later tiles
      std::vector<int32_t> tel;
      tel.reserve(owned_e.size() + halo_e.size());
      std::merge(owned_e.begin(), owned_e.end(), halo_e.begin(), halo_e.end(), std::back_inserter(tel), by_int);
      rec.own_elem_lo =
          owned_e.empty() ? 0
                          : int32_t(std::lower_bound(tel.begin(), tel.end(), owned_e.front(), by_int) - tel.begin());
      rec.n_telem = int32_t(tel.size());
      rec.telem_begin = int32_t(te_gid.size());
      // local node numbering: owned first, then halo by internal id
      std::vector<int32_t> halo_nodes;
      for (int32_t e : tel)
        for (int q = 0; q < 3; ++q) {
          int32_t u = tri[3 * e + q];
          if (node_tile[u] != gt) halo_nodes.push_back(node_int[u]);
        }
      std::sort(halo_nodes.begin(), halo_nodes.end());
      halo_nodes.erase(std::unique(halo_nodes.begin(), halo_nodes.end()), halo_nodes.end());
      rec.n_halo = int32_t(halo_nodes.size());
      rec.halo_begin = int32_t(halo_idx.size());
      if (rec.n_own + rec.n_halo > 65535 || 3 * rec.n_telem > 65535) {
        delete m;
        return fail(PF_ERR_MESH, "tile too large for 16-bit local indices; lower tile_nodes");
      }
      for (int32_t hn : halo_nodes) halo_idx.push_back(node_off + hn);
      auto local = [&](int32_t u) -> int32_t {
        if (node_tile[u] == gt) return node_int[u] - node_cursor;
        auto it = std::lower_bound(halo_nodes.begin(), halo_nodes.end(), node_int[u]);
        return rec.n_own + int32_t(it - halo_nodes.begin());
      };
      for (int32_t j = 0; j < rec.n_telem; ++j) {
        int32_t e = tel[j];
        for (int q = 0; q < 3; ++q) lc[q].push_back(uint16_t(local(tri[3 * e + q])));
        te_gid.push_back(elem_off + elem_int[e]);
        for (int q = 0; q < 6; ++q) geo_te[q].push_back(geo[e].g[q]);
        geo_te[6].push_back(geo[e].area);
      }
      // corner lists of owned nodes, ascending internal element id
      for (int32_t i = 0; i < rec.n_own; ++i) {
        int32_t u = own_user[i];
        std::vector<std::pair<int32_t, int32_t>> cs;   // (internal elem id, corner id)
        for (int32_t j = adj_ptr[u]; j < adj_ptr[u + 1]; ++j) {
          int32_t e = adj[j];
          const int32_t pos = int32_t(std::lower_bound(tel.begin(), tel.end(), e, by_int) - tel.begin());
          int q = (tri[3 * e] == u) ? 0 : (tri[3 * e + 1] == u ? 1 : 2);
          cs.emplace_back(elem_int[e], 3 * pos + q);
        }
        std::sort(cs.begin(), cs.end());
        lrow[rec.node_begin + i + 1] = int32_t(cs.size());
        for (auto& c : cs) lcorner.push_back(uint16_t(c.second));
      }
      m->max_tile_nodes = std::max(m->max_tile_nodes, rec.n_own + rec.n_halo);
      m->max_tile_elems = std::max(m->max_tile_elems, rec.n_telem);
      m->max_own = std::max(m->max_own, rec.n_own);
      m->tiles_h.push_back(rec);
      node_cursor += rec.n_own;
    }
    pf_instance_info_t& info = m->info[k];
    info.node_offset = node_off;
    info.n_nodes = n;
    info.elem_offset = elem_off;
    info.n_elems = ne;
    info.tile_offset = tile0;
    info.n_tiles = nt;
    info.h_min = hmin;
    info.area = area_sum;
    node_off += n;
    elem_off += ne;
  }
  for (int64_t i = 0; i < n_tot; ++i) lrow[i + 1] += lrow[i];
  for (TileRec& t : m->tiles_h) {
    t.corner_begin = lrow[t.node_begin];
    t.n_corner = lrow[t.node_begin + t.n_own] - t.corner_begin;
    m->max_corner = std::max(m->max_corner, t.n_corner);
  }
  m->n_tiles = int32_t(m->tiles_h.size());
  m->n_te = int32_t(te_gid.size());

  // ---- self-check of every index the kernels will use ---------------------
  {
    std::string bad;
    int32_t covered = 0;
    for (size_t ti = 0; ti < m->tiles_h.size() && bad.empty(); ++ti) {
      const TileRec& t = m->tiles_h[ti];
      const int32_t nloc = t.n_own + t.n_halo;
      if (t.node_begin != covered) bad = "owned node ranges are not contiguous";
      covered += t.n_own;
      if (t.n_own < 1 || t.n_own > kMaxTileNodes) bad = "owned node count out of range";
      if (t.halo_begin < 0 || int64_t(t.halo_begin) + t.n_halo > int64_t(halo_idx.size())) bad = "halo range";
      if (t.telem_begin < 0 || int64_t(t.telem_begin) + t.n_telem > int64_t(m->n_te)) bad = "element range";
      if (t.n_own_elem > t.n_telem || t.own_elem_begin < 0 || t.own_elem_begin + t.n_own_elem > m->n_elems ||
          t.own_elem_lo < 0 || t.own_elem_lo + t.n_own_elem > t.n_telem)
        bad = "owned element range";
      for (int32_t j = 0; j < t.n_halo && bad.empty(); ++j) {
        int32_t g = halo_idx[t.halo_begin + j];
        if (g < 0 || g >= m->n_nodes || (g >= t.node_begin && g < t.node_begin + t.n_own)) bad = "halo node id";
      }
      for (int32_t e = 0; e < t.n_telem && bad.empty(); ++e) {
        const int32_t te = t.telem_begin + e;
        if (lc[0][te] >= nloc || lc[1][te] >= nloc || lc[2][te] >= nloc) bad = "local connectivity";
        if (te_gid[te] < 0 || te_gid[te] >= m->n_elems) bad = "element id";
        if (e >= t.own_elem_lo && e < t.own_elem_lo + t.n_own_elem && te_gid[te] != t.own_elem_begin + e - t.own_elem_lo)
          bad = "owned element id";
        if (e > 0 && te_gid[te] <= te_gid[te - 1]) bad = "element order";
      }
      for (int32_t i = 0; i < t.n_own && bad.empty(); ++i) {
        const int32_t g = t.node_begin + i;
        if (lrow[g + 1] < lrow[g] || lrow[g + 1] - lrow[g] < 1) bad = "corner list";
        for (int32_t j = lrow[g]; j < lrow[g + 1] && bad.empty(); ++j)
          if (lcorner[j] >= 3 * t.n_telem || (j > lrow[g] && lcorner[j] <= lcorner[j - 1])) bad = "corner id";
      }
      // the kernels stage the corner lists in LDS with 16-bit offsets
      if (bad.empty() && (t.n_corner < t.n_own || t.n_corner > 65535 || t.corner_begin != lrow[t.node_begin] ||
                          t.corner_begin + t.n_corner != lrow[t.node_begin + t.n_own]))
        bad = "tile corner range";
    }
    if (bad.empty() && covered != m->n_nodes) bad = "tiles do not cover the nodes";
    if (bad.empty() && lrow[n_tot] != int32_t(lcorner.size())) bad = "corner list size";
    if (!bad.empty()) {
      delete m;
      return fail(PF_ERR_MESH, "internal tile-plan check failed: " + bad);
    }
  }

  // ---- device upload --------------------------------------------------------
  pf_status_t st;
  const size_t w = elem_size(dtype);
  std::vector<unsigned char> tmp;
  void *p_tiles, *p_halo, *p_lc0, *p_lc1, *p_lc2, *p_gid, *p_geo, *p_lrow, *p_lcorner, *p_invw, *p_wl, *p_fixed;
  std::vector<double> geo_all;
  geo_all.reserve(size_t(m->n_te) * 7);
  for (int q = 0; q < 7; ++q) geo_all.insert(geo_all.end(), geo_te[q].begin(), geo_te[q].end());
  // off-diagonal entries of the element stiffness K^e_kl = A_e grad phi_k . grad phi_l
  // (pairs 01, 02, 12); the rows of K^e sum to zero, so these three define it
  const size_t nte_h = size_t(m->n_te);
  std::vector<double> kw_all(3 * nte_h);
  for (size_t i = 0; i < nte_h; ++i) {
    const double A = geo_te[6][i];
    const double g0x = geo_te[0][i], g0y = geo_te[1][i], g1x = geo_te[2][i], g1y = geo_te[3][i];
    const double g2x = geo_te[4][i], g2y = geo_te[5][i];
    kw_all[i] = A * (g0x * g1x + g0y * g1y);
    kw_all[nte_h + i] = A * (g0x * g2x + g0y * g2y);
    kw_all[2 * nte_h + i] = A * (g1x * g2x + g1y * g2y);
  }
  void* p_kw;
#define UP(vec, ptr)                                  \
  if ((st = dev_upload(m, vec, &ptr)) != PF_OK) {     \
    free_all(m);                                      \
    delete m;                                         \
    return st;                                        \
  }
  UP(m->tiles_h, p_tiles);
  UP(halo_idx, p_halo);
  UP(lc[0], p_lc0);
  UP(lc[1], p_lc1);
  UP(lc[2], p_lc2);
  UP(te_gid, p_gid);
  if (dtype == PF_F64) to_dtype<double>(geo_all, tmp); else to_dtype<float>(geo_all, tmp);
  UP(tmp, p_geo);
  if (dtype == PF_F64) to_dtype<double>(kw_all, tmp); else to_dtype<float>(kw_all, tmp);
  UP(tmp, p_kw);
  UP(lrow, p_lrow);
  UP(lcorner, p_lcorner);
  if (dtype == PF_F64) to_dtype<double>(inv_w, tmp); else to_dtype<float>(inv_w, tmp);
  UP(tmp, p_invw);
  if (dtype == PF_F64) to_dtype<double>(wl, tmp); else to_dtype<float>(wl, tmp);
  UP(tmp, p_wl);
  UP(fixed, p_fixed);
#undef UP
  m->dm.tiles = static_cast<const TileRec*>(p_tiles);
  m->dm.halo_idx = static_cast<const int32_t*>(p_halo);
  m->dm.lc0 = static_cast<const uint16_t*>(p_lc0);
  m->dm.lc1 = static_cast<const uint16_t*>(p_lc1);
  m->dm.lc2 = static_cast<const uint16_t*>(p_lc2);
  m->dm.te_gid = static_cast<const int32_t*>(p_gid);
  m->dm.geo = p_geo;
  m->dm.kw = p_kw;
  m->dm.lrow = static_cast<const int32_t*>(p_lrow);
  m->dm.lcorner = static_cast<const uint16_t*>(p_lcorner);
  m->dm.inv_w = p_invw;
  m->dm.wlump = p_wl;
  m->dm.fixed = static_cast<const uint8_t*>(p_fixed);
  m->dm.n_nodes = m->n_nodes;
  m->dm.n_elems = m->n_elems;
  m->dm.n_tiles = m->n_tiles;
  m->dm.n_te = m->n_te;

  // workspaces
  const size_t nb = size_t(m->n_nodes) * w;
  void** vecs[] = {&m->dw.b,  &m->dw.dinv, &m->dw.r0, &m->dw.r1,  &m->dw.w0,  &m->dw.w1,
                   &m->dw.s0, &m->dw.s1,   &m->dw.p,  &m->dw.xw0, &m->dw.xw1, &m->dw.lam,
                   &m->dw.lam_prev, &m->dw.zb, &m->dw.y0, &m->dw.y1, &m->dw.dv};
  for (void** v : vecs)
    if ((st = dev_alloc(m, nb, v)) != PF_OK) { free_all(m); delete m; return st; }
  void* tmpp;
  if ((st = dev_alloc(m, size_t(m->n_elems) * w, &m->dw.hbar)) != PF_OK) { free_all(m); delete m; return st; }
  if ((st = dev_alloc(m, size_t(m->n_te) * w, &m->dw.mte)) != PF_OK) { free_all(m); delete m; return st; }
  if ((st = dev_alloc(m, 2 * size_t(m->n_nodes), &tmpp)) != PF_OK) { free_all(m); delete m; return st; }
  m->dw.wset = static_cast<uint8_t*>(tmpp);
  if ((st = dev_alloc(m, size_t(m->n_tiles) * 8 * sizeof(double), &tmpp)) != PF_OK) { free_all(m); delete m; return st; }
  m->dw.part = static_cast<double*>(tmpp);
  if ((st = dev_alloc(m, size_t(n_instances) * sizeof(Ctl), &tmpp)) != PF_OK) { free_all(m); delete m; return st; }
  m->dw.ctl = static_cast<Ctl*>(tmpp);
  const size_t psz = (dtype == PF_F64) ? sizeof(InstP<double>) : sizeof(InstP<float>);
  if ((st = dev_alloc(m, size_t(n_instances) * psz, &m->dw.instp)) != PF_OK) { free_all(m); delete m; return st; }
  if ((st = dev_alloc(m, size_t(n_instances) * sizeof(int), &tmpp)) != PF_OK) { free_all(m); delete m; return st; }
  m->dw.bounds = static_cast<int*>(tmpp);
  m->instp_host.assign(size_t(n_instances) * psz, 0);
  m->bounds_host.assign(size_t(n_instances), -1);
  m->params_valid = false;
  {
    hipError_t e = hipHostMalloc((void**)&m->ctl_pinned, sizeof(Ctl) * n_instances, hipHostMallocDefault);
    if (e != hipSuccess) { free_all(m); delete m; return hip_fail(e, "hipHostMalloc"); }
    e = hipEventCreateWithFlags(&m->poll_ev, hipEventDisableTiming);
    if (e != hipSuccess) { free_all(m); delete m; return hip_fail(e, "hipEventCreateWithFlags"); }
  }
  // tile counts per instance into the control blocks, and the arrival counters
  {
    std::vector<Ctl> c(n_instances);
    std::memset(c.data(), 0, sizeof(Ctl) * n_instances);
    int32_t ncnt = 0;
    for (int k = 0; k < n_instances; ++k) {
      c[k].ntiles = m->info[k].n_tiles;
      c[k].tile0 = m->info[k].tile_offset;
      c[k].nnodes = m->info[k].n_nodes;
      c[k].mode = MODE_DONE;
      c[k].ngroup = (c[k].ntiles + kArriveGroup - 1) / kArriveGroup;
      m->max_inst_tiles = std::max(m->max_inst_tiles, c[k].ntiles);
      c[k].cbase = ncnt;
      ncnt += c[k].ngroup + 1;
    }
    const size_t cbytes = size_t(ncnt) * kArriveStride * sizeof(uint32_t);
    if ((st = dev_alloc(m, cbytes, &tmpp)) != PF_OK) { free_all(m); delete m; return st; }
    m->dw.arrive = static_cast<uint32_t*>(tmpp);
    hipError_t ez = hipMemset(m->dw.arrive, 0, cbytes);
    if (ez != hipSuccess) { free_all(m); delete m; return hip_fail(ez, "hipMemset"); }
    hipError_t e = hipMemcpy(m->dw.ctl, c.data(), sizeof(Ctl) * n_instances, hipMemcpyHostToDevice);
    if (e != hipSuccess) { free_all(m); delete m; return hip_fail(e, "hipMemcpy"); }
  }
  // LDS needs: explicit = 3 node values + 6 corner values; damage = 1 node
  // value + 3 corner values of width w (its FP64 and set-up passes chunk)
  int32_t max_loc = 0, max_te = 0;
  for (const TileRec& t : m->tiles_h) {
    max_loc = std::max(max_loc, t.n_own + t.n_halo);
    max_te = std::max(max_te, t.n_telem);
  }
  // plus, in both, the owned nodes' corner lists (16-bit offsets and ids)
  const size_t lists = 2 * (size_t(m->max_own) + 1 + size_t(m->max_corner));
  m->max_lds_explicit = int32_t((3 * size_t(max_loc) + 6 * size_t(max_te)) * w + lists + 64);
  m->max_lds_explicit2 = int32_t((3 * size_t(max_loc) + 6 * ((size_t(max_te) + 1) / 2)) * w + lists + 64);
  m->max_lds_damage = int32_t(((size_t(max_loc) * w + lists + 7) & ~size_t(7)) + size_t(max_te) * 3 * w + 64);
  m->max_lds_damage2 =
      int32_t(((size_t(max_loc) * w + lists + 7) & ~size_t(7)) + ((size_t(max_te) + 1) / 2) * 3 * w + 64);
  int dev = 0, lds_limit = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds_limit <= 0)
    lds_limit = 65536;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && v > 0)
      m->lds_per_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) == hipSuccess && v > 0)
      m->threads_per_cu = v;
  }
  if (std::max(m->max_lds_explicit, m->max_lds_damage) > lds_limit) {
    std::string s = "tiles need " + std::to_string(std::max(m->max_lds_explicit, m->max_lds_damage)) +
                    " bytes of LDS, device allows " + std::to_string(lds_limit) + "; lower tile_nodes";
    free_all(m);
    delete m;
    return fail(PF_ERR_UNSUPPORTED, s);
  }
  m->device = dev;
  damage_plan(m);
  // device address of the static partials of pf_energies_static on this device
  if ((st = energy_scratch_setup(dev)) != PF_OK) { free_all(m); delete m; return st; }
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) { free_all(m); delete m; return hip_fail(e, "hipStreamSynchronize"); }
  *out = m;
  return PF_OK;
}

extern "C" pf_status_t pf_mesh_destroy(pf_mesh_t m) {
  if (!m) return PF_OK;
  (void)hipDeviceSynchronize();
  free_all(m);
  delete m;
  return PF_OK;
}

extern "C" pf_status_t pf_mesh_totals(pf_mesh_t m, pf_mesh_totals_t* out) {
  if (!m || !out) return fail(PF_ERR_ARG, "NULL argument");
  out->n_instances = m->n_inst;
  out->n_nodes = m->n_nodes;
  out->n_elems = m->n_elems;
  out->n_tiles = m->n_tiles;
  out->dtype = m->dtype;
  out->max_tile_nodes = m->max_tile_nodes;
  out->max_tile_elems = m->max_tile_elems;
  out->tile_elems_total = m->n_te;
  out->device_bytes = m->device_bytes;
  out->damage_chunks = m->dmg_nch;
  return PF_OK;
}

extern "C" pf_status_t pf_mesh_instance(pf_mesh_t m, int32_t inst, pf_instance_info_t* out) {
  if (!m || !out) return fail(PF_ERR_ARG, "NULL argument");
  if (inst < 0 || inst >= m->n_inst) return fail(PF_ERR_ARG, "instance out of range");
  *out = m->info[inst];
  return PF_OK;
}

extern "C" pf_status_t pf_mesh_node_perm(pf_mesh_t m, int32_t* out) {
  if (!m || !out) return fail(PF_ERR_ARG, "NULL argument");
  std::memcpy(out, m->node_perm.data(), sizeof(int32_t) * m->node_perm.size());
  return PF_OK;
}

extern "C" pf_status_t pf_mesh_elem_perm(pf_mesh_t m, int32_t* out) {
  if (!m || !out) return fail(PF_ERR_ARG, "NULL argument");
  std::memcpy(out, m->elem_perm.data(), sizeof(int32_t) * m->elem_perm.size());
  return PF_OK;
}

extern "C" pf_status_t pf_cfl_dt(pf_mesh_t m, const pf_params_t* p, double factor, double* dt_out) {
  if (!m || !dt_out) return fail(PF_ERR_ARG, "NULL argument");
  if (!(factor > 0) || !std::isfinite(factor)) return fail(PF_ERR_ARG, "factor must be > 0");
  pf_status_t st = check_params(m, p, nullptr, false);
  if (st != PF_OK) return st;
  for (int k = 0; k < m->n_inst; ++k) {
    const pf_params_t& q = p[k];
    const double mu = q.E / (2.0 * (1.0 + q.nu));
    const double lam = (q.plane == PF_PLANE_STRESS) ? q.E * q.nu / (1.0 - q.nu * q.nu)
                                                    : q.E * q.nu / ((1.0 + q.nu) * (1.0 - 2.0 * q.nu));
    const double cp = std::sqrt((lam + 2.0 * mu) / q.rho);
    dt_out[k] = factor * m->info[k].h_min / cp;
  }
  return PF_OK;
}

extern "C" pf_status_t pf_subcycle_limit(pf_mesh_t m, const pf_params_t* p, int32_t* n_max_out, double* ratio_out) {
  if (!m || !n_max_out) return fail(PF_ERR_ARG, "NULL argument");
  pf_status_t st = check_params(m, p, nullptr, false);
  if (st != PF_OK) return st;
  for (int k = 0; k < m->n_inst; ++k) {
    const pf_params_t& q = p[k];
    const double mu = q.E / (2.0 * (1.0 + q.nu));
    const double lam = (q.plane == PF_PLANE_STRESS) ? q.E * q.nu / (1.0 - q.nu * q.nu)
                                                    : q.E * q.nu / ((1.0 + q.nu) * (1.0 - 2.0 * q.nu));
    const double cp = std::sqrt((lam + 2.0 * mu) / q.rho);
    const double cs = std::sqrt(mu / q.rho);
    const double kap = (cs / cp) * (cs / cp);
    // Rayleigh speed c_R = cs sqrt(eta): eta is the root in (0, 1) of the
    // rationalised Rayleigh equation eta^3 - 8 eta^2 + (24 - 16 kap) eta - 16 (1 - kap) = 0
    // (negative at 0, +1 at 1), found by bisection
    auto g = [kap](double e) { return ((e - 8.0) * e + (24.0 - 16.0 * kap)) * e - 16.0 * (1.0 - kap); };
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
      const double mid = 0.5 * (lo + hi);
      (g(mid) < 0.0 ? lo : hi) = mid;
    }
    const double cr = cs * std::sqrt(0.5 * (lo + hi));
    const double ratio = cp / (0.6 * cr);
    n_max_out[k] = int32_t(std::floor(ratio));
    if (ratio_out) ratio_out[k] = ratio;
  }
  return PF_OK;
}

extern "C" pf_status_t pf_timer_enable(pf_mesh_t m, int32_t on) {
  if (!m) return fail(PF_ERR_ARG, "NULL handle");
  m->timing = on != 0;
  return PF_OK;
}

extern "C" pf_status_t pf_timer_read(pf_mesh_t m, int32_t family, double* total_ms, int64_t* launches) {
  if (!m || !total_ms || !launches) return fail(PF_ERR_ARG, "NULL argument");
  if (family < 0 || family > 4) return fail(PF_ERR_ARG, "family must be 0..4");
  Timer& t = m->timers[family];
  if (t.used) {
    PF_HIP(hipEventSynchronize(t.ev[2 * t.used - 1]));
    for (size_t k = 0; k < t.used; ++k) {
      float ms = 0.f;
      PF_HIP(hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]));
      t.ms += ms;
    }
  }
  *total_ms = t.ms;
  *launches = t.launches;
  t.ms = 0.0;
  t.launches = 0;
  t.used = 0;
  return PF_OK;
}
