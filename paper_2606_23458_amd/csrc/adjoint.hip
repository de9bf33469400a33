// Reverse of one staggered step (explicit step, then damage update).
//
// Damage update, implicit rule (Sec. 4.2, eq. implicit_adjoint_linear_system):
// with F the free nodes of the realised solve and A (scaled by l0/Gc as in
// the forward solve), lambda solves A_FF lambda_F = dbar_F (nodes cut by
// min(d, 1) carry no adjoint); then
//   dL/dGc  += -(1/Gc) lambda'(gK' K d + gM' M d + gW' w)      (AT2: the
//              element term of eq. implicit_gc_l0_element_term; AT1 its analogue)
//   With a toughness field Gc_e = Gc phi_e each element's term is dL/dGc_e
//   (optionally accumulated per element) and dL/dGc sums phi_e dL/dGc_e.
//   Hbar_e  += bH sum_k lambda_k A_e/3 - cH lambda' M^e d
//   d_prev  :  nodes held at the bound get dbar_i - (A lambda)_i.
// Explicit step: hand-written reverse mode of the corrector, the node gather,
// the element forces, the split stress (split_vjp), g(d) and the predictor.
// Nodes held at 1 are fixed in the adjoint solve and pass no adjoint.
// The history maximum passes its adjoint to psi+ where psi+ > H_n, else to H_n.
#include "device_common.hpp"
#include "split.hpp"

namespace pf {

// Right-hand side and working set of the adjoint solve; warm start from the
// previous lambda, or from zero when cold (zero on held nodes).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_prep(DevMesh dm, const uint8_t* __restrict__ act,
                                                     const T* __restrict__ dbar, T* b, uint8_t* W, T* lam,
                                                     T* lam_prev, int extrap, int cold) {
  const int tile = tile_of_block(dm.n_tiles);
  const TileRec t = dm.tiles[tile];
  for (int i = threadIdx.x; i < t.n_own; i += kBlock) {
    const int g = t.node_begin + i;
    const uint8_t a = act[g];
    // nodes held at d_prev (1) or at 1 (2) are fixed in the adjoint solve
    const uint8_t w = (a & PF_ACTIVE_LOWER) ? 1 : ((a & PF_ACTIVE_UPPER) ? 2 : 0);
    W[g] = w;
    b[g] = w ? T(0) : dbar[g];
    // start from the linear extrapolation of the last two multipliers (the
    // multiplier changes smoothly from step to step), else from the last
    const T l = lam[g];
    lam[g] = (w || cold) ? T(0) : (extrap ? T(2) * l - lam_prev[g] : l);
    lam_prev[g] = l;
  }
}

// The owned nodes' corner lists are staged in LDS at kernel entry
// (stage_corners: offsets and tile-local corner ids 3 e + k, ascending element
// id), after the kernel's other LDS arrays; each node then adds its corner
// values in list order from LDS.
__host__ __device__ __forceinline__ size_t lists_offset(size_t bytes) { return (bytes + 7) & ~size_t(7); }

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_damage(DevMesh dm, const InstP<T>* __restrict__ ip, double* part, const T* __restrict__ lam,
                                                       const T* __restrict__ dnp1, const T* __restrict__ Hnp1,
                                                       const T* __restrict__ dbar, const T* __restrict__ hbar_in,
                                                       const uint8_t* __restrict__ W, T* hbar, T* dprev_bar,
                                                       double* dgc_field) {
  __shared__ double red[4 * kWaves];
  const int tile = tile_of_block(dm.n_tiles);
  const TileRec t = dm.tiles[tile];
  const InstP<T> P = ip[t.inst];
  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  T* sl = reinterpret_cast<T*>(smem);
  T* sd = sl + nloc;
  T* qc = sd + nloc;
  uint16_t* coffs = reinterpret_cast<uint16_t*>(smem + lists_offset((2 * size_t(nloc) + 3 * size_t(t.n_telem)) * sizeof(T)));
  uint16_t* clist = coffs + t.n_own + 1;
  const int tid = threadIdx.x;
  stage_corners(dm, t, coffs, clist);
  for (int i = tid; i < nloc; i += kBlock) {
    const int g = (i < t.n_own) ? t.node_begin + i : dm.halo_idx[t.halo_begin + (i - t.n_own)];
    sl[i] = lam[g];
    sd[i] = dnp1[g];
  }
  __syncthreads();
  const T* __restrict__ geo = static_cast<const T*>(dm.geo);
  const size_t nte = size_t(dm.n_te);
  const T* __restrict__ gcs = static_cast<const T*>(dm.gcs);
  double gsum = 0.0;
  for (int e = tid; e < t.n_telem; e += kBlock) {
    const int te = t.telem_begin + e;
    const int c0 = dm.lc0[te], c1 = dm.lc1[te], c2 = dm.lc2[te];
    const T g0x = geo[te], g0y = geo[nte + te], g1x = geo[2 * nte + te], g1y = geo[3 * nte + te];
    const T g2x = geo[4 * nte + te], g2y = geo[5 * nte + te], A = geo[6 * nte + te];
    const int gid = dm.te_gid[te];
    const T He = Hnp1[gid];
    const T l0v = sl[c0], l1v = sl[c1], l2v = sl[c2];
    const T glx = g0x * l0v + g1x * l1v + g2x * l2v;
    const T gly = g0y * l0v + g1y * l1v + g2y * l2v;
    const T ls = l0v + l1v + l2v;
    const T ph = gcs ? gcs[te] : T(1);
    const T kA = P.kap * ph * A;
    const T mA = (P.c0 * ph + P.cH * He) * A * T(1.0 / 12.0);
    qc[3 * e + 0] = kA * (g0x * glx + g0y * gly) + mA * (l0v + ls);
    qc[3 * e + 1] = kA * (g1x * glx + g1y * gly) + mA * (l1v + ls);
    qc[3 * e + 2] = kA * (g2x * glx + g2y * gly) + mA * (l2v + ls);
    if (e >= t.own_elem_lo && e < t.own_elem_lo + t.n_own_elem) {
      const T d0 = sd[c0], d1 = sd[c1], d2 = sd[c2];
      const T gdx = g0x * d0 + g1x * d1 + g2x * d2;
      const T gdy = g0y * d0 + g1y * d1 + g2y * d2;
      const T ds = d0 + d1 + d2;
      const double lKd = double(A) * (double(glx) * double(gdx) + double(gly) * double(gdy));
      const double lMd = double(A) / 12.0 *
                         (double(l0v) * double(d0) + double(l1v) * double(d1) + double(l2v) * double(d2) +
                          double(ls) * double(ds));
      const double lw = double(A) / 3.0 * double(ls);
      // dL/dGc_e of this element; the instance's Gc scales every Gc_e by phi_e
      const double ge = -(double(P.gK) * lKd + double(P.gM) * lMd + double(P.gW) * lw);
      gsum += gcs ? double(ph) * ge : ge;
      if (dgc_field) dgc_field[gid] += ge;
      hbar[gid] = hbar_in[gid] + T(double(P.bH) * lw - double(P.cH) * lMd);
    }
  }
  __syncthreads();
  for (int i = tid; i < t.n_own; i += kBlock) {
    const int g = t.node_begin + i;
    T qi = T(0);
    for (int j = coffs[i]; j < coffs[i + 1]; ++j) qi += qc[clist[j]];
    dprev_bar[g] = (W[g] == 1) ? dbar[g] - qi : T(0);
  }
  gsum = block_sum(gsum, red);
  if (tid == 0) part[size_t(7) * dm.n_tiles + tile] = gsum;   // value-major partials, slot 7
}

// One workgroup per instance: dGc += the instance's tile partials, fixed order.
__global__ __launch_bounds__(kBlock) void k_adj_reduce(const Ctl* ctl, const double* part, int n_tiles, double* dGc) {
  __shared__ double red[4 * kWaves];
  const Ctl* c = ctl + blockIdx.x;
  double s = 0.0;
  const double* p7 = part + size_t(7) * n_tiles + c->tile0;
  for (int k = threadIdx.x; k < c->ntiles; k += kBlock) s += p7[k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) dGc[blockIdx.x] += s;
}

// The tile's elements are processed in nch chunks (1 or 2): each chunk's
// corner adjoints go to LDS, then every owned node adds the corners of that
// chunk, continuing its corner list where the previous chunk stopped (the
// list is in ascending element order, so the sums keep their order; two
// chunks halve the corner space so that more workgroups share a CU).
template <typename T, int S, int NPT>
__global__ __launch_bounds__(kBlock) void k_adj_explicit(DevMesh dm, const InstP<T>* __restrict__ ip, StateIn<T> sn,
                                                         StateIn<T> snp1, StateIn<T> adj1,
                                                         const T* __restrict__ hbar, StateOut<T> adj0, int vfix,
                                                         int nch) {
  const int tile = tile_of_block(dm.n_tiles);
  const TileRec t = dm.tiles[tile];
  const InstP<T> P = ip[t.inst];
  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  const int chs = (t.n_telem + nch - 1) / nch;   // elements per chunk
  T* sfx = reinterpret_cast<T*>(smem);   // adjoint of f_int at the tile's nodes
  T* sfy = sfx + nloc;
  T* sux = sfy + nloc;                   // u_{n+1}
  T* suy = sux + nloc;
  T* sd = suy + nloc;                    // d_n
  T* cux = sd + nloc;                    // corner adjoints of u_{n+1} (chunk)
  T* cuy = cux + 3 * chs;
  T* cdd = cuy + 3 * chs;                // adjoint of d_n per element (the same for its three corners)
  uint16_t* coffs = reinterpret_cast<uint16_t*>(smem + lists_offset((5 * size_t(nloc) + 7 * size_t(chs)) * sizeof(T)));
  uint16_t* clist = coffs + t.n_own + 1;
  const int tid = threadIdx.x;
  stage_corners(dm, t, coffs, clist);
  const T* __restrict__ invw = static_cast<const T*>(dm.inv_w);
  for (int i = tid; i < nloc; i += kBlock) {
    const int g = (i < t.n_own) ? t.node_begin + i : dm.halo_idx[t.halo_begin + (i - t.n_own)];
    const uint8_t fl = dm.fixed[g];
    const T minv = P.inv_rho * invw[g];
    // a_{n+1} feeds the output directly and v_{n+1} through dt/2
    const T atx = adj1.ax[g] + P.half_dt * adj1.vx[g];
    const T aty = adj1.ay[g] + P.half_dt * adj1.vy[g];
    sfx[i] = (fl & 1) ? T(0) : -minv * atx;
    sfy[i] = (fl & 2) ? T(0) : -minv * aty;
    sux[i] = snp1.ux[g];
    suy[i] = snp1.uy[g];
    sd[i] = sn.d[g];
  }
  // owned nodes' sums, carried across the chunks
  T ux_r[NPT], uy_r[NPT], dd_r[NPT];
  int jc[NPT];   // next corner of each owned node
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * kBlock;
    const int g = t.node_begin + min(i, t.n_own - 1);
    ux_r[r] = adj1.ux[g];
    uy_r[r] = adj1.uy[g];
    dd_r[r] = T(0);
    jc[r] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * kBlock;
    if (i < t.n_own) jc[r] = coffs[i];
  }
  const T* __restrict__ geo = static_cast<const T*>(dm.geo);
  const size_t nte = size_t(dm.n_te);
  for (int e0 = 0; e0 < t.n_telem; e0 += chs) {
    const int e1 = min(e0 + chs, t.n_telem);
    if (e0 > 0) __syncthreads();   // the previous chunk's corner adjoints have been added
    for (int e = e0 + tid; e < e1; e += kBlock) {
      const int te = t.telem_begin + e;
      const int c0 = dm.lc0[te], c1 = dm.lc1[te], c2 = dm.lc2[te];
      const T g0x = geo[te], g0y = geo[nte + te], g1x = geo[2 * nte + te], g1y = geo[3 * nte + te];
      const T g2x = geo[4 * nte + te], g2y = geo[5 * nte + te], A = geo[6 * nte + te];
      const T f0x = sfx[c0], f0y = sfy[c0], f1x = sfx[c1], f1y = sfy[c1], f2x = sfx[c2], f2y = sfy[c2];
      // f^e_k = A (sxx gkx + sxy gky, sxy gkx + syy gky)
      T sb[3];
      sb[0] = A * (f0x * g0x + f1x * g1x + f2x * g2x);
      sb[1] = A * (f0y * g0y + f1y * g1y + f2y * g2y);
      sb[2] = A * ((f0x * g0y + f0y * g0x) + (f1x * g1y + f1y * g1x) + (f2x * g2y + f2y * g2x));
      T exx, eyy, exy;
      elem_strain<T>(sux[c0], suy[c0], sux[c1], suy[c1], sux[c2], suy[c2], g0x, g0y, g1x, g1y, g2x, g2y, exx, eyy,
                     exy);
      T psi_p, sp[3], sm[3];
      split_eval<S, T>(exx, eyy, exy, P, psi_p, sp, sm);
      const T de = (sd[c0] + sd[c1] + sd[c2]) / T(3);
      const T om = T(1) - de;
      const T gd = om * om + P.eta;
      const int gid = dm.te_gid[te];
      const bool won = psi_p > sn.H[gid];
      const T hb = hbar[gid];
      T eb[3], gb;
      split_vjp<S, T>(exx, eyy, exy, gd, sb, won ? hb : T(0), P, eb, gb);
      const int l = e - e0;
      cux[3 * l + 0] = eb[0] * g0x + T(0.5) * eb[2] * g0y;
      cuy[3 * l + 0] = eb[1] * g0y + T(0.5) * eb[2] * g0x;
      cux[3 * l + 1] = eb[0] * g1x + T(0.5) * eb[2] * g1y;
      cuy[3 * l + 1] = eb[1] * g1y + T(0.5) * eb[2] * g1x;
      cux[3 * l + 2] = eb[0] * g2x + T(0.5) * eb[2] * g2y;
      cuy[3 * l + 2] = eb[1] * g2y + T(0.5) * eb[2] * g2x;
      cdd[l] = gb * (T(-2) * om) / T(3);
      if (e >= t.own_elem_lo && e < t.own_elem_lo + t.n_own_elem) adj0.H[gid] = won ? T(0) : hb;
    }
    __syncthreads();
    // each owned node adds this chunk's corners, in list order
    const int cend = 3 * e1, cbeg = 3 * e0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      if (i >= t.n_own) continue;
      const int j1 = coffs[i + 1];
      int j = jc[r];
      T ux = ux_r[r], uy = uy_r[r], dd = dd_r[r];
      for (; j < j1; ++j) {
        const int cc = clist[j];
        if (cc >= cend) break;
        ux += cux[cc - cbeg];
        uy += cuy[cc - cbeg];
        dd += cdd[cc / 3 - e0];
      }
      jc[r] = j;
      ux_r[r] = ux, uy_r[r] = uy, dd_r[r] = dd;
    }
  }
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int i = tid + r * kBlock;
    if (i >= t.n_own) continue;
    const int g = t.node_begin + i;
    const T ux = ux_r[r], uy = uy_r[r];
    const T vbx = adj1.vx[g], vby = adj1.vy[g];
    // prescribed velocities set by the loading ramp do not depend on v_n
    const uint8_t fl = vfix ? dm.fixed[g] : uint8_t(0);
    adj0.ux[g] = ux;
    adj0.uy[g] = uy;
    adj0.vx[g] = (fl & 1) ? T(0) : vbx + P.dt * ux;
    adj0.vy[g] = (fl & 2) ? T(0) : vby + P.dt * uy;
    adj0.ax[g] = P.half_dt * vbx + P.half_dt2 * ux;
    adj0.ay[g] = P.half_dt * vby + P.half_dt2 * uy;
    adj0.d[g] += dd_r[r];
  }
}

// LDS of an adjoint kernel: nv node values and ne values per element of the
// mesh dtype per tile (the largest tile of the handle), its elements taken
// nch chunks at a time, then the corner lists.
static size_t adjoint_lds(const pf_mesh_s* m, size_t nv, size_t ne, int nch = 1) {
  size_t vals = 0, lists = 0;
  for (const TileRec& tr : m->tiles_h) {
    const size_t chs = (size_t(tr.n_telem) + size_t(nch) - 1) / size_t(nch);
    vals = std::max(vals, (nv * size_t(tr.n_own + tr.n_halo) + ne * chs) * elem_size(m->dtype));
    lists = std::max(lists, 2 * (size_t(tr.n_own) + 1 + size_t(tr.n_corner)));
  }
  return lists_offset(vals) + lists + 64;
}

// LDS of the adjoint kernels and the element chunks of the explicit step's
// adjoint: two when halving the corner space in LDS lets more workgroups
// share a CU (capped by the CU's thread slots).  Chosen once per handle.
static void adjoint_plan(pf_mesh_s* m) {
  if (m->adj_chunks) return;
  const size_t l1 = adjoint_lds(m, 5, 7, 1), l2 = adjoint_lds(m, 5, 7, 2);
  const size_t cap = size_t(std::max(1, m->threads_per_cu / kBlock));
  const size_t occ1 = std::min(cap, size_t(m->lds_per_cu) / l1), occ2 = std::min(cap, size_t(m->lds_per_cu) / l2);
  m->adj_chunks = occ2 > occ1 ? 2 : 1;
  m->adj_lds_explicit = m->adj_chunks == 2 ? l2 : l1;
  m->adj_lds_damage = adjoint_lds(m, 2, 3);
}

template <typename T, int S>
static void launch_adj_explicit(pf_mesh_s* m, const InstP<T>* ip, const StateIn<T>& sn, const StateIn<T>& sn1,
                                const StateIn<T>& a1, const T* hb, const StateOut<T>& a0, int vfix, hipStream_t s) {
  const size_t lds = m->adj_lds_explicit;
  const int nch = m->adj_chunks;
  const int npt = (m->max_own + kBlock - 1) / kBlock;
  const dim3 grid(m->n_tiles), block(kBlock);
  if (npt <= 1)
    hipLaunchKernelGGL((k_adj_explicit<T, S, 1>), grid, block, lds, s, m->dm, ip, sn, sn1, a1, hb, a0, vfix, nch);
  else if (npt <= 2)
    hipLaunchKernelGGL((k_adj_explicit<T, S, 2>), grid, block, lds, s, m->dm, ip, sn, sn1, a1, hb, a0, vfix, nch);
  else if (npt <= 4)
    hipLaunchKernelGGL((k_adj_explicit<T, S, 4>), grid, block, lds, s, m->dm, ip, sn, sn1, a1, hb, a0, vfix, nch);
  else
    hipLaunchKernelGGL((k_adj_explicit<T, S, 8>), grid, block, lds, s, m->dm, ip, sn, sn1, a1, hb, a0, vfix, nch);
}

template <typename T>
static pf_status_t backward_t(pf_mesh_s* m, int split, const pf_state_t* s_n, const pf_state_t* s_np1,
                              const uint8_t* act, const pf_state_t* adj1, pf_state_t* adj0, double* dGc,
                              const pf_cg_opts_t* o, pf_cg_stats_t* stats, hipStream_t s) {
  const dim3 grid(m->n_tiles), block(kBlock);
  const InstP<T>* ip = static_cast<const InstP<T>*>(m->dw.instp);
  T* lam = static_cast<T*>(m->dw.lam);
  // start = 0: a cold start that forgets the multipliers of the handle's
  // previous calls (a reverse sweep that begins so repeats a fresh handle's bits)
  const bool cold = o->start == 0;
  if (cold) m->adj_calls = 0;
  timer_begin(m, 3, s);
  hipLaunchKernelGGL(k_adj_prep<T>, grid, block, 0, s, m->dm, act, static_cast<const T*>(adj1->d),
                     static_cast<T*>(m->dw.b), m->dw.wset, lam, static_cast<T*>(m->dw.lam_prev),
                     m->adj_calls >= 2 ? 1 : 0, cold ? 1 : 0);
  m->adj_calls += 1;
  timer_end(m, 3, s);
  PF_HIP(hipGetLastError());
  pf_cg_opts_t oa = *o;
  oa.resume = 0;   // every adjoint solve starts from its own set-up pass
  pf_status_t st = damage_cg(m, CG_LINEAR, s_np1->H, lam, lam, nullptr, nullptr, &oa, stats, s);
  if (st != PF_OK) return st;
  const size_t lds_d = m->adj_lds_damage;
  timer_begin(m, 3, s);
  hipLaunchKernelGGL(k_adj_damage<T>, grid, block, lds_d, s, m->dm, ip, m->dw.part, lam,
                     static_cast<const T*>(s_np1->d), static_cast<const T*>(s_np1->H),
                     static_cast<const T*>(adj1->d), static_cast<const T*>(adj1->H), m->dw.wset,
                     static_cast<T*>(m->dw.hbar), static_cast<T*>(adj0->d), m->dgc_field);
  hipLaunchKernelGGL(k_adj_reduce, dim3(m->n_inst), block, 0, s, m->dw.ctl, m->dw.part, m->n_tiles, dGc);
  const StateIn<T> sn = state_in<T>(s_n), sn1 = state_in<T>(s_np1), a1 = state_in<T>(adj1);
  const StateOut<T> a0 = state_out<T>(adj0);
  const T* hb = static_cast<const T*>(m->dw.hbar);
  const int vfix = m->ld.vfull != nullptr;
  switch (split) {
    case SPLIT_NONE: launch_adj_explicit<T, SPLIT_NONE>(m, ip, sn, sn1, a1, hb, a0, vfix, s); break;
    case SPLIT_SPECTRAL: launch_adj_explicit<T, SPLIT_SPECTRAL>(m, ip, sn, sn1, a1, hb, a0, vfix, s); break;
    case SPLIT_VOLDEV: launch_adj_explicit<T, SPLIT_VOLDEV>(m, ip, sn, sn1, a1, hb, a0, vfix, s); break;
    default: launch_adj_explicit<T, SPLIT_STAR>(m, ip, sn, sn1, a1, hb, a0, vfix, s);
  }
  timer_end(m, 3, s);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_step_backward(pf_mesh_t m, const pf_params_t* p, const double* dt, const pf_state_t* s_n,
                                        const pf_state_t* s_np1, const uint8_t* active_np1,
                                        const pf_state_t* adj_np1, pf_state_t* adj_n, double* dGc,
                                        const pf_cg_opts_t* opts, pf_cg_stats_t* stats, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  pf_status_t st;
  if ((st = check_params(m, p, dt, true)) != PF_OK) return st;
  for (int k = 0; k < m->n_inst; ++k)
    if (p[k].bounds != PF_BOUNDS_PROJECTED)
      return fail(PF_ERR_UNSUPPORTED, "the backward step supports projected bounds only");
  if (!s_n || !s_n->d || !s_n->H) return fail(PF_ERR_ARG, "s_n needs d and H");
  if (!s_np1 || !s_np1->ux || !s_np1->uy || !s_np1->d || !s_np1->H) return fail(PF_ERR_ARG, "s_np1 needs u, d and H");
  if ((st = check_state(adj_np1, true, true, "adj_np1")) != PF_OK) return st;
  if ((st = check_state(adj_n, true, true, "adj_n")) != PF_OK) return st;
  if (!active_np1 || !dGc || !opts) return fail(PF_ERR_ARG, "NULL argument");
  if (!(opts->tol > 0) || opts->max_iter < 1) return fail(PF_ERR_ARG, "need tol > 0 and max_iter >= 1");
  if (opts->precond < 0 || opts->precond > 4) return fail(PF_ERR_ARG, "precond must be in [0, 4]");
  if (states_share(adj_n, adj_np1) || states_share(adj_n, s_n) || states_share(adj_n, s_np1))
    return fail(PF_ERR_ARG, "adj_n shares an array with an input");
  adjoint_plan(m);
  const size_t lds_e = std::max(m->adj_lds_explicit, m->adj_lds_damage);
  int dev = 0, lds_limit = 65536;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds_limit = 65536;
  if (lds_e > size_t(lds_limit))
    return fail(PF_ERR_UNSUPPORTED, "tiles too large for the adjoint kernel's LDS; lower tile_nodes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  m->dt_cache.assign(dt, dt + m->n_inst);
  if ((st = upload_params(m, p, dt, s)) != PF_OK) return st;
  return (m->dtype == PF_F64)
             ? backward_t<double>(m, p[0].split, s_n, s_np1, active_np1, adj_np1, adj_n, dGc, opts, stats, s)
             : backward_t<float>(m, p[0].split, s_n, s_np1, active_np1, adj_np1, adj_n, dGc, opts, stats, s);
}
