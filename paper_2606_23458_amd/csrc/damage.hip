// Damage update (Sec. 2.2, eq. damage_pde_at2 / eq. damage_pde_at1; Sec. 2.4):
// minimise 1/2 d'Ad - b'd over d >= d_prev by a matrix-free, Jacobi-
// preconditioned projected CG, then d = min(d, 1).
//
// The system is scaled by l0/Gc (the minimiser is unchanged), so that its
// entries are of the order of the element areas in either precision; every
// dot product and scalar of the CG is accumulated in FP64.
//
// Each CG round is two launches over the tile grid:
//   A  q = A s with s = x (restart) or s = p = z + beta p_old (iteration);
//      on the first restart also assembles b and the Jacobi diagonal;
//      partial p'q and the largest feasible step along p.
//   B  restart: r = b - q, working set W, z = D^-1 r on free nodes;
//      iteration: x += alpha p (cut at the first bound hit), r -= alpha q, z.
// The last block of each instance to finish a launch combines the tiles'
// partials in a fixed order (so results are bitwise reproducible) and
// advances that instance's state machine:
//   - a step cut by a bound adds the blocking nodes to W and restarts;
//   - when the free residual max |r_i|/A_ii <= tol the solve restarts from the
//     true residual; there, nodes of W with r_i/A_ii > tol are released;
//     the solve ends when both scaled residual tests pass.
// A node enters W only at the bound with r_i < 0 (it wants to go lower).
#include "device_common.hpp"

namespace pf {

template <typename T>
struct DmgArgs {
  DevMesh dm;
  const InstP<T>* __restrict__ ip;
  Ctl* ctl;
  double* part;
  const T* __restrict__ H;
  const T* __restrict__ lb;
  T* x;
  T* b; T* dinv; T* r; T* z; T* p0; T* p1; T* q;
  uint8_t* W;
  double tol;
  int32_t max_iter;
  int32_t kind;        // CG_QP or CG_LINEAR
};

__global__ void k_dmg_init(Ctl* ctl, int n_inst, int kind) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_inst) return;
  Ctl& c = ctl[k];
  c.mode = MODE_RESTART;
  c.setup = 1;
  c.release = 0;
  c.hit = 0;
  c.iters = 0;
  c.restarts = 0;
  c.flags = 0;
  c.nact = 0;
  c.pbuf = 0;
  c.cnt_a = 0;
  c.cnt_b = 0;
  c.cnt_c = 0;
  c.rz = 0.0;
  c.alpha = 0.0;
  c.beta = 0.0;
  c.amax = 0.0;
  c.resid = 0.0;
  c.pq = 0.0;
  c.ref = (kind == CG_QP) ? 1.0 : 0.0;
}

// Largest feasible step ratio of a node moving down; computed identically in
// kernels A and B so that the blocking node is recognised exactly.
template <typename T>
__device__ __forceinline__ double step_ratio(T lbv, T xv, T pv) {
  return (double(lbv) - double(xv)) / double(pv);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_a(DmgArgs<T> a) {
  __shared__ double red[kWaves];
  __shared__ int sflag;
  const TileRec t = a.dm.tiles[blockIdx.x];
  Ctl* c = a.ctl + t.inst;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  const InstP<T> P = a.ip[t.inst];
  const bool restart = (mode == MODE_RESTART);
  const bool setup = restart && (c->setup != 0);
  const double beta = c->beta;
  const int pb = c->pbuf;
  const T* pold = pb ? a.p1 : a.p0;
  T* pnew = pb ? a.p0 : a.p1;

  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  T* s = reinterpret_cast<T*>(smem);
  T* qc = s + nloc;                 // [3 n_telem] corner values of A^e s^e
  T* dc = qc + 3 * t.n_telem;       // [3 n_telem] diagonal corners (setup)
  T* bc = dc + 3 * t.n_telem;       // [n_telem]   load per corner (setup)
  const int tid = threadIdx.x;

  for (int i = tid; i < nloc; i += kBlock) {
    const int g = (i < t.n_own) ? t.node_begin + i : a.dm.halo_idx[t.halo_begin + (i - t.n_own)];
    T v;
    if (setup && a.kind == CG_QP) {
      v = a.lb[g];
      if (i < t.n_own) a.x[g] = v;
    } else if (restart) {
      v = a.x[g];
    } else {
      const T zz = a.z[g];
      v = (beta == 0.0) ? zz : zz + T(beta) * pold[g];
      if (i < t.n_own) pnew[g] = v;
    }
    s[i] = v;
  }
  __syncthreads();

  const T* __restrict__ geo = static_cast<const T*>(a.dm.geo);
  const size_t nte = size_t(a.dm.n_te);
  for (int e = tid; e < t.n_telem; e += kBlock) {
    const int te = t.telem_begin + e;
    const int c0 = a.dm.lc0[te], c1 = a.dm.lc1[te], c2 = a.dm.lc2[te];
    const T g0x = geo[te], g0y = geo[nte + te], g1x = geo[2 * nte + te], g1y = geo[3 * nte + te];
    const T g2x = geo[4 * nte + te], g2y = geo[5 * nte + te], A = geo[6 * nte + te];
    const T He = a.H[a.dm.te_gid[te]];
    const T kA = P.kap * A;
    const T mA = (P.c0 + P.cH * He) * A * T(1.0 / 12.0);
    const T s0 = s[c0], s1 = s[c1], s2 = s[c2];
    const T gpx = g0x * s0 + g1x * s1 + g2x * s2;
    const T gpy = g0y * s0 + g1y * s1 + g2y * s2;
    const T ss = s0 + s1 + s2;
    qc[3 * e + 0] = kA * (g0x * gpx + g0y * gpy) + mA * (s0 + ss);
    qc[3 * e + 1] = kA * (g1x * gpx + g1y * gpy) + mA * (s1 + ss);
    qc[3 * e + 2] = kA * (g2x * gpx + g2y * gpy) + mA * (s2 + ss);
    if (setup) {
      dc[3 * e + 0] = kA * (g0x * g0x + g0y * g0y) + T(2) * mA;
      dc[3 * e + 1] = kA * (g1x * g1x + g1y * g1y) + T(2) * mA;
      dc[3 * e + 2] = kA * (g2x * g2x + g2y * g2y) + T(2) * mA;
      if (a.kind == CG_QP) bc[e] = (P.b0 + P.bH * He) * A * T(1.0 / 3.0);
    }
  }
  __syncthreads();

  double pq = 0.0, amin = INFINITY;
  const bool projected = (a.kind == CG_QP) && (P.bounds == PF_BOUNDS_PROJECTED);
  for (int i = tid; i < t.n_own; i += kBlock) {
    const int g = t.node_begin + i;
    const int j0 = a.dm.lrow[g], j1 = a.dm.lrow[g + 1];
    T qi = T(0);
    for (int j = j0; j < j1; ++j) qi += qc[a.dm.lcorner[j]];
    a.q[g] = qi;
    if (setup) {
      T di = T(0), bi = T(0);
      for (int j = j0; j < j1; ++j) {
        const int cc = a.dm.lcorner[j];
        di += dc[cc];
        bi += bc[cc / 3];
      }
      if (a.kind == CG_QP) a.b[g] = bi;
      a.dinv[g] = T(1) / di;
    }
    if (!restart) {
      const T pv = s[i];
      pq += double(pv) * double(qi);
      if (projected && pv < T(0) && !a.W[g]) amin = fmin(amin, step_ratio<T>(a.lb[g], a.x[g], pv));
    }
  }
  if (restart) return;   // the restart's reductions happen in kernel B

  pq = block_sum(pq, red);
  amin = block_min(amin, red);
  if (tid == 0) {
    a.part[8 * blockIdx.x + 0] = pq;
    a.part[8 * blockIdx.x + 1] = amin;
  }
  if (!arrive_last(&c->cnt_a, c->ntiles, &sflag)) return;
  double sq = 0.0, sm = INFINITY;
  for (int k = tid; k < c->ntiles; k += kBlock) {
    sq += a.part[8 * (c->tile0 + k) + 0];
    sm = fmin(sm, a.part[8 * (c->tile0 + k) + 1]);
  }
  sq = block_sum(sq, red);
  sm = block_min(sm, red);
  if (tid == 0) {
    double alpha = c->rz / sq;
    int hit = 0;
    if (!(sq > 0.0) || !isfinite(alpha)) {
      c->flags |= PF_FLAG_NONFINITE;
      c->mode = MODE_DONE;
      alpha = 0.0;
    } else if (sm <= alpha) {
      alpha = sm;
      hit = 1;
    }
    c->pq = sq;
    c->amax = sm;
    c->alpha = alpha;
    c->hit = hit;
    c->pbuf = pb ^ 1;
    c->cnt_a = 0;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_b(DmgArgs<T> a) {
  __shared__ double red[kWaves];
  __shared__ int sflag;
  const TileRec t = a.dm.tiles[blockIdx.x];
  Ctl* c = a.ctl + t.inst;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  const InstP<T> P = a.ip[t.inst];
  const bool restart = (mode == MODE_RESTART);
  const bool qp = (a.kind == CG_QP);
  const bool projected = qp && (P.bounds == PF_BOUNDS_PROJECTED);
  const double tol = a.tol;
  const int tid = threadIdx.x;
  double rz = 0.0, cf = 0.0, ca = -INFINITY, na = 0.0, rb = 0.0;
  if (restart) {
    const bool release = c->release != 0;
    const bool fresh = c->setup != 0;   // the first restart ignores the previous solve's working set
    for (int i = tid; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      const T bi = a.b[g];
      const T ri = bi - a.q[g];
      const T di = a.dinv[g];
      bool w = false;
      if (projected) {
        const bool at = a.x[g] <= a.lb[g];
        const bool keep = !fresh && a.W[g] && !(release && double(ri) * double(di) > tol);
        w = at && (ri < T(0) || keep);
      } else if (!qp) {
        w = a.W[g] != 0;
      }
      if (!qp && fresh && !w) rb = fmax(rb, fabs(double(bi) * double(di)));
      const T zi = w ? T(0) : di * ri;
      a.r[g] = ri;
      a.z[g] = zi;
      a.W[g] = w ? 1 : 0;
      rz += double(ri) * double(zi);
      const double sr = double(ri) * double(di);
      if (w) {
        ca = fmax(ca, sr);
        na += 1.0;
      } else {
        cf = fmax(cf, fabs(sr));
      }
    }
  } else {
    const double alpha = c->alpha;
    const bool hit = c->hit != 0;
    const T* p = c->pbuf ? a.p1 : a.p0;
    const T al = T(alpha);
    for (int i = tid; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      const T pv = p[g];
      const T xv = a.x[g];
      const T lbv = a.lb[g];
      bool w = a.W[g] != 0;
      T xn = xv + al * pv;
      if (projected) {
        if (hit && !w && pv < T(0) && step_ratio<T>(lbv, xv, pv) <= alpha) {
          xn = lbv;
          w = true;
          a.W[g] = 1;
        } else if (xn < lbv) {
          xn = lbv;
        }
      }
      a.x[g] = xn;
      if (!hit) {
        const T ri = a.r[g] - al * a.q[g];
        const T di = a.dinv[g];
        const T zi = w ? T(0) : di * ri;
        a.r[g] = ri;
        a.z[g] = zi;
        rz += double(ri) * double(zi);
        const double sr = double(ri) * double(di);
        if (w) {
          ca = fmax(ca, sr);
          na += 1.0;
        } else {
          cf = fmax(cf, fabs(sr));
        }
      }
    }
  }
  rz = block_sum(rz, red);
  cf = block_max(cf, red);
  ca = block_max(ca, red);
  na = block_sum(na, red);
  rb = block_max(rb, red);
  if (tid == 0) {
    double* pp = a.part + 8 * blockIdx.x;
    pp[2] = rz;
    pp[3] = cf;
    pp[4] = ca;
    pp[5] = na;
    pp[6] = rb;
  }
  if (!arrive_last(&c->cnt_b, c->ntiles, &sflag)) return;
  double srz = 0.0, scf = 0.0, sca = -INFINITY, sna = 0.0, srb = 0.0;
  for (int k = tid; k < c->ntiles; k += kBlock) {
    const double* pp = a.part + 8 * (c->tile0 + k);
    srz += pp[2];
    scf = fmax(scf, pp[3]);
    sca = fmax(sca, pp[4]);
    sna += pp[5];
    srb = fmax(srb, pp[6]);
  }
  srz = block_sum(srz, red);
  scf = block_max(scf, red);
  sca = block_max(sca, red);
  sna = block_sum(sna, red);
  srb = block_max(srb, red);
  if (tid == 0) {
    c->iters += 1;
    c->cnt_b = 0;
    if (restart && c->setup && !qp) c->ref = srb;   // linear solves stop relative to max |b_i|/A_ii
    const double tl = tol * c->ref;
    if (restart) {
      c->setup = 0;
      c->nact = int32_t(sna);
      c->resid = fmax(scf, sca) / (c->ref > 0.0 ? c->ref : 1.0);
      if (!isfinite(srz) || !isfinite(scf)) {
        c->flags |= PF_FLAG_NONFINITE;
        c->mode = MODE_DONE;
      } else if (!qp && c->ref == 0.0) {
        c->mode = MODE_DONE;   // zero right-hand side: the solution is 0 (set by the final kernel)
      } else if (scf <= tl && sca <= tl) {
        c->mode = MODE_DONE;
      } else if (scf <= tl) {
        // free set converged but held nodes want to move up: release them
        c->mode = MODE_RESTART;
        c->release = 1;
        c->restarts += 1;
      } else {
        c->mode = MODE_ITER;
        c->beta = 0.0;
        c->rz = srz;
      }
    } else if (c->hit) {
      c->mode = MODE_RESTART;
      c->release = 0;
      c->restarts += 1;
    } else {
      if (!isfinite(srz)) {
        c->flags |= PF_FLAG_NONFINITE;
        c->mode = MODE_DONE;
      } else {
        c->beta = srz / c->rz;
        c->rz = srz;
        c->resid = scf / (c->ref > 0.0 ? c->ref : 1.0);
        if (scf <= tl || srz == 0.0) {
          c->mode = MODE_RESTART;
          c->release = (sca > tl) ? 1 : 0;
          c->restarts += 1;
        }
      }
    }
    if (c->mode != MODE_DONE && c->iters >= a.max_iter) {
      c->flags |= PF_FLAG_NOT_CONVERGED;
      c->mode = MODE_DONE;
    }
  }
}

// Apply the upper bound, write the active flags and the statistics.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_final(DmgArgs<T> a, uint8_t* active_out, pf_cg_stats_t* stats) {
  const TileRec t = a.dm.tiles[blockIdx.x];
  const Ctl* c = a.ctl + t.inst;
  const InstP<T> P = a.ip[t.inst];
  const bool projected = (P.bounds == PF_BOUNDS_PROJECTED);
  if (a.kind != CG_QP) {
    if (c->ref == 0.0)
      for (int i = threadIdx.x; i < t.n_own; i += kBlock) a.x[t.node_begin + i] = T(0);
  } else
  for (int i = threadIdx.x; i < t.n_own; i += kBlock) {
    const int g = t.node_begin + i;
    T xv = a.x[g];
    const T lbv = a.lb[g];
    uint8_t act;
    if (projected) {
      act = a.W[g] ? PF_ACTIVE_LOWER : 0;
    } else {
      act = (xv < lbv) ? PF_ACTIVE_LOWER : 0;
      if (act) xv = lbv;
    }
    if (xv > T(1)) {
      xv = T(1);
      act |= PF_ACTIVE_UPPER;
    }
    a.x[g] = xv;
    if (active_out) active_out[g] = act;
  }
  if (stats && threadIdx.x == 0 && int(blockIdx.x) == c->tile0) {
    pf_cg_stats_t s;
    s.iters = c->iters;
    s.restarts = c->restarts;
    s.n_active = c->nact;
    s.flags = c->flags | (c->mode == MODE_DONE ? 0 : PF_FLAG_NOT_CONVERGED);
    s.resid = c->resid;
    stats[t.inst] = s;
  }
}

template <typename T>
static DmgArgs<T> dmg_args(pf_mesh_s* m, int kind, const void* H, const void* d_prev, void* d, double tol,
                          int max_iter) {
  DmgArgs<T> a;
  a.kind = kind;
  a.dm = m->dm;
  a.ip = static_cast<const InstP<T>*>(m->dw.instp);
  a.ctl = m->dw.ctl;
  a.part = m->dw.part;
  a.H = static_cast<const T*>(H);
  a.lb = static_cast<const T*>(d_prev);
  a.x = static_cast<T*>(d);
  a.b = static_cast<T*>(m->dw.b);
  a.dinv = static_cast<T*>(m->dw.dinv);
  a.r = static_cast<T*>(m->dw.r);
  a.z = static_cast<T*>(m->dw.z);
  a.p0 = static_cast<T*>(m->dw.p0);
  a.p1 = static_cast<T*>(m->dw.p1);
  a.q = static_cast<T*>(m->dw.q);
  a.W = m->dw.wset;
  a.tol = tol;
  a.max_iter = max_iter;
  return a;
}

// Enqueue one solve; `rounds_done` returns how many CG rounds were launched.
template <typename T>
static pf_status_t run_solve(pf_mesh_s* m, int kind, const void* H, const void* d_prev, void* d,
                             uint8_t* active_out, const pf_cg_opts_t* o, pf_cg_stats_t* stats, hipStream_t s) {
  DmgArgs<T> a = dmg_args<T>(m, kind, H, d_prev, d, o->tol, o->max_iter);
  const dim3 grid(m->n_tiles), block(kBlock);
  const size_t lds = m->max_lds_damage;
  hipLaunchKernelGGL(k_dmg_init, dim3((m->n_inst + 63) / 64), dim3(64), 0, s, m->dw.ctl, m->n_inst, kind);
  auto round = [&]() {
    timer_begin(m, 1, s);
    hipLaunchKernelGGL(k_dmg_a<T>, grid, block, lds, s, a);
    timer_end(m, 1, s);
    timer_begin(m, 2, s);
    hipLaunchKernelGGL(k_dmg_b<T>, grid, block, 0, s, a);
    timer_end(m, 2, s);
  };
  const int max_rounds = o->max_iter;
  int launched = 0;
  if (o->check_every <= 0) {
    for (; launched < max_rounds; ++launched) round();
  } else {
    int chunk = std::min(o->check_every, 4);
    while (launched < max_rounds) {
      const int n = std::min(chunk, max_rounds - launched);
      for (int k = 0; k < n; ++k) round();
      launched += n;
      PF_HIP(hipGetLastError());
      PF_HIP(hipMemcpyAsync(m->ctl_pinned, m->dw.ctl, sizeof(Ctl) * m->n_inst, hipMemcpyDeviceToHost, s));
      PF_HIP(hipStreamSynchronize(s));
      bool all_done = true;
      for (int k = 0; k < m->n_inst; ++k) all_done = all_done && (m->ctl_pinned[k].mode == MODE_DONE);
      if (all_done) break;
      chunk = std::min(2 * chunk, std::max(o->check_every, 4));
    }
  }
  hipLaunchKernelGGL(k_dmg_final<T>, grid, block, 0, s, a, active_out, stats);
  PF_HIP(hipGetLastError());
  if (o->check_every > 0) {
    PF_HIP(hipMemcpyAsync(m->ctl_pinned, m->dw.ctl, sizeof(Ctl) * m->n_inst, hipMemcpyDeviceToHost, s));
    PF_HIP(hipStreamSynchronize(s));
    int flags = 0;
    for (int k = 0; k < m->n_inst; ++k) {
      flags |= m->ctl_pinned[k].flags;
      if (m->ctl_pinned[k].mode != MODE_DONE) flags |= PF_FLAG_NOT_CONVERGED;
    }
    if (flags & PF_FLAG_NONFINITE) return fail(PF_ERR_NONFINITE, "non-finite value in the damage CG");
    if (flags & PF_FLAG_NOT_CONVERGED) return fail(PF_ERR_NOT_CONVERGED, "damage CG reached max_iter");
  }
  return PF_OK;
}

pf_status_t damage_cg(pf_mesh_s* m, int kind, const void* H, const void* lb, void* x, uint8_t* active_out,
                      const pf_cg_opts_t* o, pf_cg_stats_t* stats, hipStream_t s) {
  return (m->dtype == PF_F64) ? run_solve<double>(m, kind, H, lb, x, active_out, o, stats, s)
                              : run_solve<float>(m, kind, H, lb, x, active_out, o, stats, s);
}

}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_damage_solve(pf_mesh_t m, const pf_params_t* p, const void* H, const void* d_prev, void* d,
                                       uint8_t* active_out, const pf_cg_opts_t* opts, pf_cg_stats_t* stats,
                                       pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  pf_status_t st;
  if ((st = check_params(m, p, nullptr, false)) != PF_OK) return st;
  if (!H || !d_prev || !d || !opts) return fail(PF_ERR_ARG, "NULL argument");
  if (d == d_prev) return fail(PF_ERR_ARG, "d must not alias d_prev");
  if (!(opts->tol > 0) || opts->max_iter < 1) return fail(PF_ERR_ARG, "need tol > 0 and max_iter >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = upload_params(m, p, nullptr, s)) != PF_OK) return st;
  return damage_cg(m, CG_QP, H, d_prev, d, active_out, opts, stats, s);
}
