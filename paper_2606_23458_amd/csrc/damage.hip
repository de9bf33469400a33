// Damage update (Sec. 2.2, eq. damage_pde_at2 / eq. damage_pde_at1; Sec. 2.4):
// minimise 1/2 d'Ad - b'd over d_prev <= d <= 1 by a matrix-free, Jacobi-
// preconditioned projected CG.
//
// The system is scaled by l0/Gc (the minimiser is unchanged), so that its
// entries are of the order of the element areas in either precision; every
// dot product and scalar of the CG is accumulated in FP64.
//
// Method.  CG runs on the free nodes with the held nodes frozen at a bound
// (d_prev or 1), and the held set is updated between CG runs (Sec. 2.4:
// nodes at the lower bound with negative residual are frozen; the solver
// restarts on the updated free set).  The held set starts from the caller's
// guess (normally the previous step's flags).  After each converged CG run
// a check pass recomputes the true residual r = b - Ax, moves free nodes that
// left [d_prev, 1] onto the bound they crossed, and releases held nodes whose
// scaled residual r_i/A_ii points into the interior by more than tol; the
// solve ends when a check changes nothing and the free residual passes.
// Each check is one primal-dual active-set update; if eight updates have not
// settled the set, the solve switches to a monotone projected CG: steps are
// cut at the first bound and followed by a projected Jacobi-gradient step of
// length 0.25 (below 2/lambda_max(D^-1 A) for row sums of |A_ij|/A_ii up to
// 8), and held nodes are released only when CG on the current face has
// converged.  Nodes with d_prev = 1 are fixed.  A CG run is also cut short
// for a check when a quarter of its free nodes have left [d_prev, 1] (a far
// wrong held set, e.g. the first AT1 step, would otherwise cost a solve of a
// nearly singular free system).
//
// Each CG round is four launches: over the tile grid
//   A  q = A s with s = x (restart, check) or s = p = z + beta p_old
//      (iteration); on the first pass also assembles b and the diagonal;
//      per-tile partial p'q (and the largest feasible step, monotone flavour);
//   B  restart / check: r = b - q, held-set update, z = D^-1 r on free nodes;
//      iteration: x += alpha p, r -= alpha q, z; per-tile partials;
// and, after each, one workgroup per instance (k_dmg_reduce_a / _b) that
// combines that instance's per-tile partials in a fixed order (so results
// are bitwise reproducible) and advances the instance's state.  No atomics
// and no device-wide fences are used.  Linear mode (CG_LINEAR) solves
// A_FF x_F = b_F for a fixed held set and is used by the adjoint step.
#include "device_common.hpp"

namespace pf {

constexpr int kSwitchAfter = 8;        // active-set updates before the monotone fallback
constexpr double kExpandStep = 0.25;   // projected-gradient step of the fallback

enum { HELD_NONE = 0, HELD_LOWER = 1, HELD_UPPER = 2 };

template <typename T>
struct DmgArgs {
  DevMesh dm;
  const InstP<T>* __restrict__ ip;
  Ctl* ctl;
  double* part;
  const T* __restrict__ H;
  const T* __restrict__ lb;
  const uint8_t* __restrict__ guess;
  T* x;                // the iterate (a workspace for the damage solve)
  T* dout;             // damage solve: output array (read at set-up when start = 1)
  T* mte;              // per-solve mass coefficient of each tile element
  T* b; T* dinv; T* r; T* z; T* p0; T* p1; T* q;
  uint8_t* W;
  double tol;
  int32_t max_iter;
  int32_t kind;        // CG_QP or CG_LINEAR
  int32_t start;       // 1: extrapolated start for the damage solve
};

__global__ void k_dmg_init(Ctl* ctl, int n_inst, int kind, int monotone) {
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
  c.flavor = (kind == CG_QP && monotone) ? 1 : 0;
  c.outer = 0;
  c.inner = 0;
  c.rz = 0.0;
  c.alpha = 0.0;
  c.beta = 0.0;
  c.amax = 0.0;
  c.resid = 0.0;
  c.pq = 0.0;
  c.ref = (kind == CG_QP) ? 1.0 : 0.0;
}

template <typename T>
__device__ __forceinline__ T clamp01(T v, T lo) {
  return v < lo ? lo : (v > T(1) ? T(1) : v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_a(DmgArgs<T> a) {
  __shared__ double red[kWaves];
  const TileRec t = a.dm.tiles[blockIdx.x];
  const Ctl* c = a.ctl + t.inst;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  const InstP<T> P = a.ip[t.inst];
  const bool matvec_x = (mode != MODE_ITER);
  const bool setup = matvec_x && (c->setup != 0);
  const bool qp = (a.kind == CG_QP);
  const bool projected = qp && (P.bounds == PF_BOUNDS_PROJECTED);
  const bool monotone = projected && (c->flavor != 0);
  const double beta = c->beta;
  const int pb = c->pbuf;
  const T* pold = pb ? a.p1 : a.p0;
  T* pnew = pb ? a.p0 : a.p1;

  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  T* s = reinterpret_cast<T*>(smem);
  T* qc = s + nloc;                 // [3 n_telem] corner values of A^e s^e
  T* dc = qc + 3 * t.n_telem;       // [3 n_telem] diagonal corners (first pass)
  T* bc = dc + 3 * t.n_telem;       // [n_telem]   load per corner (first pass, QP)
  const int tid = threadIdx.x;

  for (int i = tid; i < nloc; i += kBlock) {
    const int g = (i < t.n_own) ? t.node_begin + i : a.dm.halo_idx[t.halo_begin + (i - t.n_own)];
    T v;
    if (setup && qp) {
      // start at d_prev (or its extrapolation in time), or at 1 where the guess
      // holds the node at the upper bound
      const T lbv = a.lb[g];
      if (projected && a.guess && (a.guess[g] & PF_ACTIVE_UPPER)) {
        v = T(1);
      } else if (a.start) {
        v = clamp01<T>(T(2) * lbv - a.dout[g], lbv);
      } else {
        v = lbv;
      }
      if (i < t.n_own) a.x[g] = v;
    } else if (matvec_x) {
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
    const T kA = P.kap * A;
    T mA, He = T(0);
    if (setup) {
      He = a.H[a.dm.te_gid[te]];
      mA = (P.c0 + P.cH * He) * A * T(1.0 / 12.0);
      a.mte[te] = mA;
    } else {
      mA = a.mte[te];
    }
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
      bc[e] = qp ? (P.b0 + P.bH * He) * A * T(1.0 / 3.0) : T(0);
    }
  }
  __syncthreads();

  double pq = 0.0, amin = INFINITY;
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
      if (qp) a.b[g] = bi;
      a.dinv[g] = T(1) / di;
    }
    if (!matvec_x) {
      const T pv = s[i];
      pq += double(pv) * double(qi);
      if (monotone && a.W[g] == HELD_NONE) {
        // largest step that keeps this node inside [d_prev, 1]
        if (pv < T(0)) amin = fmin(amin, (double(a.lb[g]) - double(a.x[g])) / double(pv));
        if (pv > T(0)) amin = fmin(amin, (1.0 - double(a.x[g])) / double(pv));
      }
    }
  }
  if (matvec_x) return;   // restart and check passes reduce in kernel B
  pq = block_sum(pq, red);
  amin = block_min(amin, red);
  if (tid == 0) {
    a.part[8 * blockIdx.x + 0] = pq;
    a.part[8 * blockIdx.x + 1] = amin;
  }
}

// One workgroup per instance: step length of the current iteration.
__global__ __launch_bounds__(kBlock) void k_dmg_reduce_a(Ctl* ctl, const double* part) {
  __shared__ double red[kWaves];
  Ctl* c = ctl + blockIdx.x;
  if (c->mode != MODE_ITER) return;
  double sq = 0.0, sm = INFINITY;
  for (int k = threadIdx.x; k < c->ntiles; k += kBlock) {
    sq += part[8 * (c->tile0 + k) + 0];
    sm = fmin(sm, part[8 * (c->tile0 + k) + 1]);
  }
  sq = block_sum(sq, red);
  sm = block_min(sm, red);
  if (threadIdx.x != 0) return;
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
  c->pbuf ^= 1;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_b(DmgArgs<T> a) {
  __shared__ double red[kWaves];
  const TileRec t = a.dm.tiles[blockIdx.x];
  const Ctl* c = a.ctl + t.inst;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  const InstP<T> P = a.ip[t.inst];
  const bool qp = (a.kind == CG_QP);
  const bool projected = qp && (P.bounds == PF_BOUNDS_PROJECTED);
  const bool monotone = projected && (c->flavor != 0);
  const bool setup = c->setup != 0;
  const double tol = a.tol;
  const int tid = threadIdx.x;
  // partials: rz, max free |r|/A_ii, max held "wants to leave" r/A_ii, held count, max |b|/A_ii, changes
  double rz = 0.0, cf = 0.0, ca = -INFINITY, na = 0.0, rb = 0.0, ch = 0.0;
  if (mode != MODE_ITER) {
    const bool release = c->release != 0;
    for (int i = tid; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      const T bi = a.b[g];
      const T ri = bi - a.q[g];
      const T di = a.dinv[g];
      const double sr = double(ri) * double(di);
      uint8_t w = HELD_NONE;
      if (!qp) {
        w = a.W[g];
        if (setup && w == HELD_NONE) rb = fmax(rb, fabs(double(bi) * double(di)));
      } else if (projected) {
        const T xv = a.x[g], lbv = a.lb[g];
        const uint8_t wold = a.W[g];
        if (lbv >= T(1)) {
          w = HELD_LOWER;   // d_prev = 1: the node is fixed
        } else if (mode == MODE_CHECK) {
          const bool viol_lo = wold == HELD_NONE && double(lbv) - double(xv) > tol;
          const bool viol_up = wold == HELD_NONE && double(xv) - 1.0 > tol;
          const bool rel = (wold == HELD_LOWER && sr > tol) || (wold == HELD_UPPER && sr < -tol);
          w = viol_lo ? HELD_LOWER : (viol_up ? HELD_UPPER : (rel ? HELD_NONE : wold));
          if (viol_lo) a.x[g] = lbv;
          if (viol_up) a.x[g] = T(1);
          ch += (viol_lo || viol_up || rel) ? 1.0 : 0.0;
        } else if (setup) {
          const uint8_t gs = a.guess ? a.guess[g] : uint8_t(0);
          w = ((gs & PF_ACTIVE_LOWER) && xv <= lbv) ? HELD_LOWER
                                                    : (((gs & PF_ACTIVE_UPPER) && xv >= T(1)) ? HELD_UPPER : HELD_NONE);
        } else if (!monotone) {
          w = wold;
        } else {
          const bool want_lo = ri < T(0) || (wold == HELD_LOWER && !(release && sr > tol));
          const bool want_up = ri > T(0) || (wold == HELD_UPPER && !(release && sr < -tol));
          w = (xv <= lbv && want_lo) ? HELD_LOWER : ((xv >= T(1) && want_up) ? HELD_UPPER : HELD_NONE);
        }
      }
      const T zi = w ? T(0) : di * ri;
      a.r[g] = ri;
      a.z[g] = zi;
      a.W[g] = w;
      rz += double(ri) * double(zi);
      if (w) {
        ca = fmax(ca, w == HELD_UPPER ? -sr : sr);
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
      const uint8_t w = a.W[g];
      const T qv = a.q[g];
      const T di = a.dinv[g];
      if (hit) {
        // monotone flavour: step to the first bound, then a projected Jacobi-gradient step
        if (!w) {
          const T xh = xv + al * pv;
          const T rh = a.r[g] - al * qv;
          a.x[g] = clamp01<T>(xh + T(kExpandStep) * di * rh, a.lb[g]);
        }
        continue;
      }
      T xn = xv + al * pv;
      if (monotone) {
        xn = clamp01<T>(xn, a.lb[g]);
      } else if (projected && !w) {
        const double xd = double(xn);
        if (double(a.lb[g]) - xd > tol || xd - 1.0 > tol) ch += 1.0;   // free node outside the bounds
      }
      a.x[g] = xn;
      const T ri = a.r[g] - al * qv;
      const T zi = w ? T(0) : di * ri;
      a.r[g] = ri;
      a.z[g] = zi;
      rz += double(ri) * double(zi);
      const double sr = double(ri) * double(di);
      if (w) {
        ca = fmax(ca, w == HELD_UPPER ? -sr : sr);
      } else {
        cf = fmax(cf, fabs(sr));
      }
    }
  }
  rz = block_sum(rz, red);
  cf = block_max(cf, red);
  ca = block_max(ca, red);
  na = block_sum(na, red);
  rb = block_max(rb, red);
  ch = block_sum(ch, red);
  if (tid == 0) {
    double* pp = a.part + 8 * blockIdx.x;
    pp[2] = rz;
    pp[3] = cf;
    pp[4] = ca;
    pp[5] = na;
    pp[6] = rb;
    pp[7] = ch;
  }
}

// One workgroup per instance: combine kernel B's partials and advance the state.
__global__ __launch_bounds__(kBlock) void k_dmg_reduce_b(Ctl* ctl, const double* part, const int* bounds, int kind,
                                                         double tol, int max_iter) {
  __shared__ double red[kWaves];
  Ctl* c = ctl + blockIdx.x;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  double srz = 0.0, scf = 0.0, sca = -INFINITY, sna = 0.0, srb = 0.0, sch = 0.0;
  for (int k = threadIdx.x; k < c->ntiles; k += kBlock) {
    const double* pp = part + 8 * (c->tile0 + k);
    srz += pp[2];
    scf = fmax(scf, pp[3]);
    sca = fmax(sca, pp[4]);
    sna += pp[5];
    srb = fmax(srb, pp[6]);
    sch += pp[7];
  }
  srz = block_sum(srz, red);
  scf = block_max(scf, red);
  sca = block_max(sca, red);
  sna = block_sum(sna, red);
  srb = block_max(srb, red);
  sch = block_sum(sch, red);
  if (threadIdx.x != 0) return;
  const bool qp = (kind == CG_QP);
  const bool projected = qp && (bounds[blockIdx.x] == PF_BOUNDS_PROJECTED);
  const bool monotone = projected && (c->flavor != 0);
  const bool setup = c->setup != 0;
  c->iters += 1;
  c->inner = (mode == MODE_ITER) ? c->inner + 1 : 0;
  if (setup && !qp) c->ref = srb;   // linear solves stop relative to max |b_i|/A_ii
  const double tl = tol * c->ref;
  const double rs = c->ref > 0.0 ? c->ref : 1.0;
  if (mode != MODE_ITER) {
    c->setup = 0;
    c->nact = int32_t(sna);
    c->resid = (monotone ? fmax(scf, sca) : scf) / rs;
    if (!isfinite(srz) || !isfinite(scf)) {
      c->flags |= PF_FLAG_NONFINITE;
      c->mode = MODE_DONE;
    } else if (!qp && c->ref == 0.0) {
      c->mode = MODE_DONE;   // zero right-hand side: the solution is 0 (set by the final kernel)
    } else if (mode == MODE_CHECK) {
      if (sch > 0.0) {
        c->outer += 1;
        c->restarts += 1;
        if (c->outer >= kSwitchAfter) c->flavor = 1;
        c->release = 0;
        c->mode = MODE_RESTART;
      } else if (scf <= tl) {
        c->mode = MODE_DONE;
      } else {
        c->mode = MODE_ITER;
        c->beta = 0.0;
        c->rz = srz;
      }
    } else if (monotone) {
      if (scf <= tl && sca <= tl) {
        c->mode = MODE_DONE;
      } else if (scf <= tl) {
        c->mode = MODE_RESTART;   // face converged, held nodes want to leave: release them
        c->release = 1;
        c->restarts += 1;
      } else {
        c->mode = MODE_ITER;
        c->beta = 0.0;
        c->rz = srz;
      }
    } else if (scf <= tl) {
      c->mode = projected ? MODE_CHECK : MODE_DONE;
    } else {
      c->mode = MODE_ITER;
      c->beta = 0.0;
      c->rz = srz;
    }
  } else if (c->hit) {
    c->mode = MODE_RESTART;
    c->release = 0;
    c->restarts += 1;
  } else if (!isfinite(srz)) {
    c->flags |= PF_FLAG_NONFINITE;
    c->mode = MODE_DONE;
  } else {
    c->beta = srz / c->rz;
    c->rz = srz;
    c->resid = scf / rs;
    const bool early = projected && !monotone && c->inner >= 2 && sch > 0.25 * double(c->nnodes - c->nact);
    if (scf <= tl || srz == 0.0 || early) {
      // this CG run converged on its recurrence residual, or a quarter of the
      // free nodes already left their bounds: update the held set now
      if (projected && !monotone) {
        c->mode = MODE_CHECK;
      } else {
        c->mode = MODE_RESTART;
        c->release = (monotone && sca > tl) ? 1 : 0;
        c->restarts += monotone ? 1 : 0;
      }
    }
  }
  if (c->mode != MODE_DONE && c->iters >= max_iter) {
    c->flags |= PF_FLAG_NOT_CONVERGED;
    c->mode = MODE_DONE;
  }
}

// Final pass: bounds, active flags and statistics.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_final(DmgArgs<T> a, uint8_t* active_out, pf_cg_stats_t* stats) {
  const TileRec t = a.dm.tiles[blockIdx.x];
  const Ctl* c = a.ctl + t.inst;
  const InstP<T> P = a.ip[t.inst];
  const bool projected = (P.bounds == PF_BOUNDS_PROJECTED);
  if (a.kind != CG_QP) {
    if (c->ref == 0.0)
      for (int i = threadIdx.x; i < t.n_own; i += kBlock) a.x[t.node_begin + i] = T(0);
  } else {
    for (int i = threadIdx.x; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      T xv = a.x[g];
      const T lbv = a.lb[g];
      uint8_t act = 0;
      if (projected) {
        const uint8_t w = a.W[g];
        act = (w == HELD_LOWER) ? PF_ACTIVE_LOWER : ((w == HELD_UPPER) ? PF_ACTIVE_UPPER : 0);
        xv = clamp01<T>(xv, lbv);   // free nodes within tol outside the bounds
      } else {
        if (xv < lbv) {
          xv = lbv;
          act = PF_ACTIVE_LOWER;
        }
        if (xv > T(1)) {
          xv = T(1);
          act |= PF_ACTIVE_UPPER;
        }
      }
      a.dout[g] = xv;
      if (active_out) active_out[g] = act;
    }
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
static DmgArgs<T> dmg_args(pf_mesh_s* m, int kind, const void* H, const void* d_prev, void* d,
                           const uint8_t* guess, double tol, int max_iter, int start) {
  DmgArgs<T> a;
  a.kind = kind;
  a.start = (kind == CG_QP) ? start : 0;
  a.mte = static_cast<T*>(m->dw.mte);
  a.dm = m->dm;
  a.ip = static_cast<const InstP<T>*>(m->dw.instp);
  a.ctl = m->dw.ctl;
  a.part = m->dw.part;
  a.H = static_cast<const T*>(H);
  a.lb = static_cast<const T*>(d_prev);
  a.guess = guess;
  // the damage solve iterates in a workspace and writes d at the end; linear solves iterate in place
  a.x = (kind == CG_QP) ? static_cast<T*>(m->dw.xw) : static_cast<T*>(d);
  a.dout = static_cast<T*>(d);
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

template <typename T>
static pf_status_t run_solve(pf_mesh_s* m, int kind, const void* H, const void* d_prev, void* d,
                             const uint8_t* guess, uint8_t* active_out, const pf_cg_opts_t* o,
                             pf_cg_stats_t* stats, hipStream_t s) {
  DmgArgs<T> a = dmg_args<T>(m, kind, H, d_prev, d, guess, o->tol, o->max_iter, o->start);
  const dim3 grid(m->n_tiles), block(kBlock), igrid(m->n_inst);
  const size_t lds = m->max_lds_damage;
  hipLaunchKernelGGL(k_dmg_init, dim3((m->n_inst + 63) / 64), dim3(64), 0, s, m->dw.ctl, m->n_inst, kind, o->monotone);
  auto round = [&]() {
    timer_begin(m, 1, s);
    hipLaunchKernelGGL(k_dmg_a<T>, grid, block, lds, s, a);
    timer_end(m, 1, s);
    timer_begin(m, 4, s);
    hipLaunchKernelGGL(k_dmg_reduce_a, igrid, block, 0, s, m->dw.ctl, m->dw.part);
    timer_end(m, 4, s);
    timer_begin(m, 2, s);
    hipLaunchKernelGGL(k_dmg_b<T>, grid, block, 0, s, a);
    timer_end(m, 2, s);
    timer_begin(m, 4, s);
    hipLaunchKernelGGL(k_dmg_reduce_b, igrid, block, 0, s, m->dw.ctl, m->dw.part, m->dw.bounds, kind, o->tol,
                       o->max_iter);
    timer_end(m, 4, s);
  };
  const int max_rounds = o->max_iter;
  int launched = 0;
  if (o->check_every <= 0) {
    for (; launched < max_rounds; ++launched) round();
  } else {
    int chunk = std::min(o->check_every, 8);
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
      chunk = std::max(chunk, o->check_every);
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

pf_status_t damage_cg(pf_mesh_s* m, int kind, const void* H, const void* lb, void* x, const uint8_t* guess,
                      uint8_t* active_out, const pf_cg_opts_t* o, pf_cg_stats_t* stats, hipStream_t s) {
  return (m->dtype == PF_F64) ? run_solve<double>(m, kind, H, lb, x, guess, active_out, o, stats, s)
                              : run_solve<float>(m, kind, H, lb, x, guess, active_out, o, stats, s);
}

}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_damage_solve(pf_mesh_t m, const pf_params_t* p, const void* H, const void* d_prev, void* d,
                                       const uint8_t* active_guess, uint8_t* active_out, const pf_cg_opts_t* opts,
                                       pf_cg_stats_t* stats, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  pf_status_t st;
  if ((st = check_params(m, p, nullptr, false)) != PF_OK) return st;
  if (!H || !d_prev || !d || !opts) return fail(PF_ERR_ARG, "NULL argument");
  if (d == d_prev) return fail(PF_ERR_ARG, "d must not alias d_prev");
  if (!(opts->tol > 0) || opts->max_iter < 1) return fail(PF_ERR_ARG, "need tol > 0 and max_iter >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = upload_params(m, p, nullptr, s)) != PF_OK) return st;
  return damage_cg(m, CG_QP, H, d_prev, d, active_guess, active_out, opts, stats, s);
}
