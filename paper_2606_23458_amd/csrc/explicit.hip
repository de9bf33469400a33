// Explicit step (Sec. 2.2-2.3): velocity-Verlet predictor, P1 strain, energy
// split with degradation, element forces, deterministic node gather,
// corrector and the history maximum -- fused into one tile kernel.
//
// One workgroup per tile.  Phase 1 forms the predictor u* = u + dt v + dt^2/2 a
// for the tile's owned and halo nodes in LDS (owned nodes also write u_{n+1}).
// Phase 2 evaluates every element touching an owned node and stores its three
// corner forces in LDS; owned elements also update H.  Phase 3 sums, for each
// owned node, its corner forces in ascending element order (no atomics, so
// the result is bitwise reproducible) and applies the corrector.  Phases 2
// and 3 may run over the tile's elements in two chunks, which halves the
// corner-force space in LDS so that more workgroups fit on a CU; a node's
// corner list is sorted by element, so each chunk adds a contiguous run of
// it and the sums keep their order.
//
// Ramped loads (pf_set_loading) are evaluated per workgroup from the state
// time t_n: the traction factor S(t_{n+1}) scales the registered nodal force
// and the velocity factor R(t_n + dt/2) the prescribed velocities.
#include <cmath>

#include "device_common.hpp"
#include "split.hpp"

namespace pf {

// Smooth traction ramp of Sec. 3 (eq. smooth_traction_ramp): 0 before t = 0,
// half a cosine wave up to t_r, then 1.
__device__ __forceinline__ double ramp_smooth(double t, double t_r) {
  if (t <= 0.0) return 0.0;
  if (t_r <= 0.0 || t >= t_r) return 1.0;
  return 0.5 * (1.0 - cos(M_PI * (t / t_r)));
}

// Linear velocity ramp of Sec. 3 (eq. kalthoff_velocity_ramp), as a fraction
// of the full velocity.
__device__ __forceinline__ double ramp_linear(double t, double t_v) {
  if (t_v <= 0.0 || t >= t_v) return 1.0;
  return t > 0.0 ? t / t_v : 0.0;
}

template <typename T, int S, int NPT, int BS>
__global__ __launch_bounds__(BS) void k_explicit(DevMesh dm, const InstP<T>* __restrict__ ip, StateIn<T> in,
                                                 StateOut<T> out, const T* __restrict__ fext, int nch, LoadDev ld,
                                                 const double* __restrict__ tin, double* __restrict__ tout) {
  const int tile = tile_of_block(dm.n_tiles);
  const TileRec t = dm.tiles[tile];
  const InstP<T> P = ip[t.inst];
  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  const int chs = (t.n_telem + nch - 1) / nch;   // elements per chunk
  T* sux = reinterpret_cast<T*>(smem);
  T* suy = sux + nloc;
  T* sd = suy + nloc;
  T* sfx = sd + nloc;
  T* sfy = sfx + 3 * chs;
  uint16_t* coffs = reinterpret_cast<uint16_t*>(sfy + 3 * chs);         // [n_own + 1] corner-list offsets
  uint16_t* clist = coffs + t.n_own + 1;                                // [n_corner] corner ids
  const int tid = threadIdx.x;
  // corner-list loads first (registers), stored to LDS after the predictor
  StagedCorners<(BS == 256 ? 2 : 1), (BS == 256 ? 12 : 6)> scn;
  stage_corners_load(dm, t, scn);
  // so are each thread's first halo node id and first element record
  // (clamped on threads past the end)
  const int hg0 = t.n_halo > 0 ? dm.halo_idx[t.halo_begin + min(tid, t.n_halo - 1)] : t.node_begin;
  const T* __restrict__ geo = static_cast<const T*>(dm.geo);
  const size_t nte = size_t(dm.n_te);
  const int pte = t.telem_begin + min(tid, t.n_telem - 1);
  const int pc0 = dm.lc0[pte], pc1 = dm.lc1[pte], pc2 = dm.lc2[pte];
  T pg[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) pg[k] = geo[size_t(k) * nte + pte];

  // ramped loads: the force factor S(t_{n+1}) and the prescribed velocities
  // R(t_n + dt/2) v_full (the same values in every thread of the workgroup)
  T fsc = T(1), vsc = T(1);
  const T* __restrict__ vfull = nullptr;
  if (ld.par) {
    const double tn = tin[t.inst];
    const LoadP lp = ld.par[t.inst];
    fext = static_cast<const T*>(ld.F);
    vfull = static_cast<const T*>(ld.vfull);
    fsc = T(ramp_smooth(tn + P.dtd, lp.t_f));
    vsc = T(ramp_linear(tn + 0.5 * P.dtd, lp.t_v));
  }

  // ---- phase 1: predictor (eq. vv_u) -------------------------------------
  // the corrector's inputs (lumped mass, prescribed flags, external force)
  // are loaded here too, so that the last phase waits on no memory
  const T* __restrict__ invw = static_cast<const T*>(dm.inv_w);
  const size_t N = size_t(dm.n_nodes);
  T rvx[NPT], rvy[NPT], rax[NPT], ray[NPT], rmi[NPT], rex[NPT], rey[NPT];
  uint8_t rfl[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * BS;
    if (i < t.n_own) {
      const int g = t.node_begin + i;
      rmi[r] = invw[g];
      rfl[r] = dm.fixed[g];
      rex[r] = fext ? fsc * fext[g] : T(0);
      rey[r] = fext ? fsc * fext[N + g] : T(0);
      T vx = in.vx[g], vy = in.vy[g];
      const T ax = in.ax[g], ay = in.ay[g];
      if (vfull) {
        if (rfl[r] & 1) vx = vsc * vfull[g];
        if (rfl[r] & 2) vy = vsc * vfull[N + g];
      }
      const T usx = in.ux[g] + P.dt * vx + P.half_dt2 * ax;
      const T usy = in.uy[g] + P.dt * vy + P.half_dt2 * ay;
      sux[i] = usx;
      suy[i] = usy;
      sd[i] = in.d[g];
      out.ux[g] = usx;
      out.uy[g] = usy;
      rvx[r] = vx, rvy[r] = vy, rax[r] = ax, ray[r] = ay;
    }
  }
  auto halo = [&](int i, int g) {
    T vx = in.vx[g], vy = in.vy[g];
    if (vfull) {
      const uint8_t fl = dm.fixed[g];
      if (fl & 1) vx = vsc * vfull[g];
      if (fl & 2) vy = vsc * vfull[N + g];
    }
    sux[i] = in.ux[g] + P.dt * vx + P.half_dt2 * in.ax[g];
    suy[i] = in.uy[g] + P.dt * vy + P.half_dt2 * in.ay[g];
    sd[i] = in.d[g];
  };
  if (tid < t.n_halo) halo(t.n_own + tid, hg0);
  for (int i = t.n_own + BS + tid; i < nloc; i += BS) halo(i, dm.halo_idx[t.halo_begin + (i - t.n_own)]);
  stage_corners_store(dm, t, scn, coffs, clist);
  __syncthreads();

  // ---- phases 2 and 3a, per chunk of elements ------------------------------
  T fxa[NPT], fya[NPT];
  int jc[NPT];   // next corner of each owned node
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * BS;
    fxa[r] = T(0), fya[r] = T(0);
    jc[r] = (i < t.n_own) ? coffs[i] : 0;
  }
  for (int e0 = 0; e0 < t.n_telem; e0 += chs) {
  const int e1 = min(e0 + chs, t.n_telem);
  if (e0 > 0) __syncthreads();   // the previous chunk's corner forces have been added
  // phase 2: element strain, split, stress, corner forces, history
  auto element = [&](int e, int c0, int c1, int c2, T g0x, T g0y, T g1x, T g1y, T g2x, T g2y, T A) {
    const T u0x = sux[c0], u0y = suy[c0], u1x = sux[c1], u1y = suy[c1], u2x = sux[c2], u2y = suy[c2];
    T exx, eyy, exy;
    elem_strain<T>(u0x, u0y, u1x, u1y, u2x, u2y, g0x, g0y, g1x, g1y, g2x, g2y, exx, eyy, exy);
    T psi_p, sp[3], sm[3];
    split_eval<S, T>(exx, eyy, exy, P, psi_p, sp, sm);
    const T de = (sd[c0] + sd[c1] + sd[c2]) / T(3);
    const T om = T(1) - de;
    const T gd = om * om + P.eta;
    const T sxx = gd * sp[0] + sm[0], syy = gd * sp[1] + sm[1], sxy = gd * sp[2] + sm[2];
    const int l = e - e0;
    sfx[3 * l + 0] = A * (sxx * g0x + sxy * g0y);
    sfy[3 * l + 0] = A * (sxy * g0x + syy * g0y);
    sfx[3 * l + 1] = A * (sxx * g1x + sxy * g1y);
    sfy[3 * l + 1] = A * (sxy * g1x + syy * g1y);
    sfx[3 * l + 2] = A * (sxx * g2x + sxy * g2y);
    sfy[3 * l + 2] = A * (sxy * g2x + syy * g2y);
    if (e >= t.own_elem_lo && e < t.own_elem_lo + t.n_own_elem) {
      const int gid = t.own_elem_begin + (e - t.own_elem_lo);
      const T Hn = in.H[gid];
      out.H[gid] = psi_p > Hn ? psi_p : Hn;
    }
  };
  int e = e0 + tid;
  if (e0 == 0 && e < e1) {
    // this thread's first element, loaded at kernel entry
    element(e, pc0, pc1, pc2, pg[0], pg[1], pg[2], pg[3], pg[4], pg[5], pg[6]);
    e += BS;
  }
  for (; e < e1; e += BS) {
    const int te = t.telem_begin + e;
    element(e, dm.lc0[te], dm.lc1[te], dm.lc2[te], geo[te], geo[nte + te], geo[2 * nte + te], geo[3 * nte + te],
            geo[4 * nte + te], geo[5 * nte + te], geo[6 * nte + te]);
  }
  __syncthreads();
  // phase 3a: each owned node adds the corners of this chunk, in list order
  const int cend = 3 * e1, cbeg = 3 * e0;
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * BS;
    if (i < t.n_own) {
      const int j1 = coffs[i + 1];
      int j = jc[r];
      T fx = fxa[r], fy = fya[r];
      for (; j < j1; ++j) {
        const int c = clist[j];
        if (c >= cend) break;
        fx += sfx[c - cbeg];
        fy += sfy[c - cbeg];
      }
      jc[r] = j;
      fxa[r] = fx, fya[r] = fy;
    }
  }
  }

  // ---- phase 3b: corrector (eq. vv_a, eq. vv_v) ----------------------------
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * BS;
    if (i < t.n_own) {
      const int g = t.node_begin + i;
      const T fx = fxa[r], fy = fya[r];
      const T minv = P.inv_rho * rmi[r];
      const uint8_t fl = rfl[r];
      const T ex = rex[r];
      const T ey = rey[r];
      const T axn = (fl & 1) ? T(0) : minv * (ex - fx);
      const T ayn = (fl & 2) ? T(0) : minv * (ey - fy);
      out.vx[g] = rvx[r] + P.half_dt * (rax[r] + axn);
      out.vy[g] = rvy[r] + P.half_dt * (ray[r] + ayn);
      out.ax[g] = axn;
      out.ay[g] = ayn;
    }
  }
  // the state time, advanced once per instance (by its first tile)
  if (tout && tid == 0 && (tile == 0 || dm.tiles[tile - 1].inst != t.inst)) tout[t.inst] = tin[t.inst] + P.dtd;
}

// Two element chunks when that lets more workgroups share a CU (LDS-bound
// occupancy); the workgroups per CU are capped by the CU's thread slots.
static int explicit_chunks(const pf_mesh_s* m, int bs) {
  if (m->explicit_chunks > 0) return m->explicit_chunks;
  const int cap = std::max(1, m->threads_per_cu / bs);
  const int occ1 = std::min(cap, m->lds_per_cu / std::max(1, m->max_lds_explicit));
  const int occ2 = std::min(cap, m->lds_per_cu / std::max(1, m->max_lds_explicit2));
  return occ2 > occ1 ? 2 : 1;
}

template <typename T, int S>
static hipError_t launch_explicit_s(pf_mesh_s* m, const pf_state_t* in, pf_state_t* out, const void* fext,
                                    hipStream_t s) {
  const LoadDev ld = m->ld;
  const double* tin = in->t;
  double* tout = (in->t && out->t) ? out->t : nullptr;
  const int nch = explicit_chunks(m, m->explicit_block);
  const size_t lds = nch == 2 ? m->max_lds_explicit2 : m->max_lds_explicit;
  const InstP<T>* ip = static_cast<const InstP<T>*>(m->dw.instp);
  auto si = state_in<T>(in);
  auto so = state_out<T>(out);
  const T* fe = static_cast<const T*>(fext);
  const dim3 grid(m->n_tiles);
  if (m->explicit_block == 512) {
    const int npt = (m->max_own + 511) / 512;
    if (npt <= 1)
      hipLaunchKernelGGL((k_explicit<T, S, 1, 512>), grid, dim3(512), lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
    else if (npt <= 2)
      hipLaunchKernelGGL((k_explicit<T, S, 2, 512>), grid, dim3(512), lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
    else
      hipLaunchKernelGGL((k_explicit<T, S, 4, 512>), grid, dim3(512), lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
  } else {
    const int npt = (m->max_own + kBlock - 1) / kBlock;
    const dim3 block(kBlock);
    if (npt <= 1)
      hipLaunchKernelGGL((k_explicit<T, S, 1, kBlock>), grid, block, lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
    else if (npt <= 2)
      hipLaunchKernelGGL((k_explicit<T, S, 2, kBlock>), grid, block, lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
    else if (npt <= 4)
      hipLaunchKernelGGL((k_explicit<T, S, 4, kBlock>), grid, block, lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
    else
      hipLaunchKernelGGL((k_explicit<T, S, 8, kBlock>), grid, block, lds, s, m->dm, ip, si, so, fe, nch, ld, tin, tout);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_explicit(pf_mesh_s* m, int split, const pf_state_t* in, pf_state_t* out, const void* fext,
                                  hipStream_t s) {
  switch (split) {
    case SPLIT_NONE: return launch_explicit_s<T, SPLIT_NONE>(m, in, out, fext, s);
    case SPLIT_SPECTRAL: return launch_explicit_s<T, SPLIT_SPECTRAL>(m, in, out, fext, s);
    case SPLIT_VOLDEV: return launch_explicit_s<T, SPLIT_VOLDEV>(m, in, out, fext, s);
    default: return launch_explicit_s<T, SPLIT_STAR>(m, in, out, fext, s);
  }
}

pf_status_t check_state(const pf_state_t* s, bool need_d, bool need_H, const char* name) {
  if (!s) return fail(PF_ERR_ARG, std::string(name) + " is NULL");
  const void* p[] = {s->ux, s->uy, s->vx, s->vy, s->ax, s->ay};
  for (const void* q : p)
    if (!q) return fail(PF_ERR_ARG, std::string(name) + " has a NULL array");
  if (need_d && !s->d) return fail(PF_ERR_ARG, std::string(name) + ".d is NULL");
  if (need_H && !s->H) return fail(PF_ERR_ARG, std::string(name) + ".H is NULL");
  return PF_OK;
}

bool states_share(const pf_state_t* a, const pf_state_t* b) {
  const void* pa[] = {a->ux, a->uy, a->vx, a->vy, a->ax, a->ay, a->d, a->H};
  const void* pb[] = {b->ux, b->uy, b->vx, b->vy, b->ax, b->ay, b->d, b->H};
  for (const void* x : pa)
    for (const void* y : pb)
      if (x && x == y) return true;
  return false;
}

}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_explicit_step(pf_mesh_t m, const pf_params_t* p, const double* dt, const pf_state_t* in,
                                        pf_state_t* out, const void* f_ext, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  pf_status_t st;
  if ((st = check_params(m, p, dt, true)) != PF_OK) return st;
  if ((st = check_state(in, true, true, "in")) != PF_OK) return st;
  if ((st = check_state(out, false, true, "out")) != PF_OK) return st;
  if (states_share(in, out)) return fail(PF_ERR_ARG, "in and out share an array");
  if (in->t && in->t == out->t) return fail(PF_ERR_ARG, "in and out share the time array");
  if (m->ld.par) {
    if (!in->t || !out->t) return fail(PF_ERR_ARG, "ramped loads are registered: in->t and out->t are required");
    if (f_ext) return fail(PF_ERR_ARG, "ramped loads are registered: f_ext must be NULL");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  m->dt_cache.assign(dt, dt + m->n_inst);
  if ((st = upload_params(m, p, dt, s)) != PF_OK) return st;
  timer_begin(m, 0, s);
  hipError_t e = (m->dtype == PF_F64) ? launch_explicit<double>(m, p[0].split, in, out, f_ext, s)
                                      : launch_explicit<float>(m, p[0].split, in, out, f_ext, s);
  timer_end(m, 0, s);
  if (e != hipSuccess) return hip_fail(e, "k_explicit launch");
  return PF_OK;
}

namespace pf {

template <typename T>
static pf_status_t check_finite(const void* a, size_t n, hipStream_t s, const char* name) {
  std::vector<T> h(n);
  PF_HIP(hipMemcpyAsync(h.data(), a, n * sizeof(T), hipMemcpyDeviceToHost, s));
  PF_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(double(h[i]))) return fail(PF_ERR_ARG, std::string(name) + " has a non-finite entry");
  return PF_OK;
}

}  // namespace pf

extern "C" pf_status_t pf_set_loading(pf_mesh_t m, const void* F, const void* v_full, const double* t_traction,
                                      const double* t_velocity, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!F && !v_full) {
    m->ld = LoadDev{};
    return PF_OK;
  }
  std::vector<LoadP> lp(size_t(m->n_inst));
  for (int k = 0; k < m->n_inst; ++k) {
    lp[size_t(k)].t_f = t_traction ? t_traction[k] : 0.0;
    lp[size_t(k)].t_v = t_velocity ? t_velocity[k] : 0.0;
    if (!std::isfinite(lp[size_t(k)].t_f) || !std::isfinite(lp[size_t(k)].t_v))
      return fail(PF_ERR_ARG, "instance " + std::to_string(k) + ": ramp times must be finite");
  }
  const bool f64 = m->dtype == PF_F64;
  const size_t vec = 2 * size_t(m->n_nodes) * (f64 ? sizeof(double) : sizeof(float));
  for (const void* a : {F, v_full}) {
    if (!a) continue;
    const pf_status_t st = f64 ? check_finite<double>(a, 2 * size_t(m->n_nodes), s, a == F ? "F" : "v_full")
                               : check_finite<float>(a, 2 * size_t(m->n_nodes), s, a == F ? "F" : "v_full");
    if (st != PF_OK) return st;
  }
  const size_t off_v = (vec + 255) / 256 * 256;
  const size_t off_p = off_v + off_v;
  if (!m->load_buf) {
    void* p = nullptr;
    const size_t bytes = off_p + sizeof(LoadP) * size_t(m->n_inst);
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(PF_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    m->allocs.push_back(p);   // freed with the handle
    m->device_bytes += bytes;
    m->load_buf = p;
  }
  char* base = static_cast<char*>(m->load_buf);
  // nothing enqueued earlier on the stream may still read the previous loads
  PF_HIP(hipStreamSynchronize(s));
  if (F) PF_HIP(hipMemcpyAsync(base, F, vec, hipMemcpyDeviceToDevice, s));
  if (v_full) PF_HIP(hipMemcpyAsync(base + off_v, v_full, vec, hipMemcpyDeviceToDevice, s));
  PF_HIP(hipMemcpyAsync(base + off_p, lp.data(), sizeof(LoadP) * lp.size(), hipMemcpyHostToDevice, s));
  PF_HIP(hipStreamSynchronize(s));
  m->ld.F = F ? base : nullptr;
  m->ld.vfull = v_full ? base + off_v : nullptr;
  m->ld.par = reinterpret_cast<const LoadP*>(base + off_p);
  return PF_OK;
}
