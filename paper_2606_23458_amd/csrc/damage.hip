// Damage update (Sec. 2.2, eq. damage_pde_at2 / eq. damage_pde_at1; Sec. 2.4):
// minimise 1/2 d'Ad - b'd over d_prev <= d <= 1 by a matrix-free, Jacobi-
// preconditioned projected CG.
//
// The system is scaled by l0/Gc (the minimiser is unchanged), so that its
// entries are of the order of the element areas in either precision; every
// dot product and scalar of the CG is accumulated in FP64.
//
// Method.  CG runs on the free nodes with the held nodes frozen at a bound
// (d_prev or 1), and the held set is updated between CG runs, the bound
// treatment of Sec. 2.4 organised as primal-dual active-set steps.  The held
// set starts from the caller's
// guess (normally the previous step's flags).  After each converged CG run
// a check pass recomputes the true residual r = b - Ax, moves free nodes that
// left [d_prev, 1] onto the bound they crossed, and releases held nodes whose
// scaled residual r_i/A_ii points into the interior by more than tol/4; the
// solve ends when a check changes nothing and the free residual passes.
// (With a release threshold near tol, where the solution's tail varies on the
// scale of tol, each release pushes the next ring of held nodes just over the
// threshold and the held set shrinks one ring per check; well below tol the
// whole tail is released at once.)  A restart pass sees the state a check
// would see and counts the changes that check would make: a restart whose
// free residual passes with none to make ends the solve (a damage field that
// does not move, e.g. AT1 below its threshold, takes one round).
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
// Iteration.  The CG recurrences are arranged so that one iteration needs a
// single reduction (the Chronopoulos-Gear form): with z = M r (M = D^-1 on
// free nodes, 0 on held ones), w = A z and s = A p,
//     p = z + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//     z = M r,  w = A z,  gamma = r'z,  delta = z'w,
//     beta' = gamma'/gamma,  alpha' = gamma'/(delta' - beta' gamma'/alpha).
// One round of the solve is one or two launches over the tile grid:
//   k_dmg      one pass of the current phase for every tile of every
//              instance that is not done:
//                restart / check: x-matvec in FP64, true residual, held-set
//                  update (the first restart also assembles b, the diagonal
//                  and the per-solve mass coefficients);
//                first: z = M r and w = A z of a new CG run;
//                iterate: the vector updates above and w = A z, where each
//                  tile recomputes z on its halo nodes from the previous
//                  vectors, so no second pass is needed;
//              and per-tile partial sums.  A pass takes its tile's elements
//              in one or two chunks (the corner values of a chunk in LDS,
//              each owned node adding them in its corner-list order), two
//              where that lets every workgroup of the pass be resident at
//              once (damage_chunks);
//   k_dmg_red  one workgroup per instance combines its tiles' partials in a
//              fixed order (bitwise reproducible results) and advances the
//              instance's state.
// With the Jacobi preconditioner and instances of up to kFuseMaxTiles tiles
// the combination instead runs at the end of k_dmg, in the instance's last
// workgroup to finish (arrivals counted by integer atomics; same order, same
// bits), so such a round is a single launch.
// r, w, s and x are ping-pong pairs: a pass reads one half and writes the
// other, so halo reads never race with the owners' writes.  No floating-point
// atomics and no device-wide fences are used.  Linear mode (CG_LINEAR) solves
// A_FF x_F = b_F for a fixed held set and is used by the adjoint step.
#include <climits>
#include <cstring>

#include "device_common.hpp"

namespace pf {

constexpr int kSwitchAfter = 8;        // active-set updates before the monotone fallback
constexpr double kExpandStep = 0.25;   // projected-gradient step of the fallback
constexpr double kRelease = 0.25;      // held nodes are released when their scaled residual
                                       // points inward by more than kRelease * tol

// held-set states; HELD_FIXED: d_prev = 1, the node cannot move
enum { HELD_NONE = 0, HELD_LOWER = 1, HELD_UPPER = 2, HELD_FIXED = 3 };

// partial sums of one tile, and how each combines (2 bits each: 0 sum, 1 min, 2 max)
enum { PT_DELTA = 0, PT_AMIN = 1, PT_GAMMA = 2, PT_CF = 3, PT_CA = 4, PT_NA = 5, PT_RB = 6, PT_CH = 7 };
constexpr uint32_t kPartOps = (0u << 0) | (1u << 2) | (0u << 4) | (2u << 6) | (2u << 8) | (0u << 10) | (2u << 12) |
                              (0u << 14);

template <typename T>
struct DmgArgs {
  DevMesh dm;
  const InstP<T>* __restrict__ ip;
  Ctl* ctl;
  double* part;
  const T* __restrict__ H;
  const T* __restrict__ lb;
  const uint8_t* __restrict__ guess;
  T* x0; T* x1;        // iterate pair (QP: workspaces; linear: the caller's x and a workspace)
  T* r0; T* r1;        // residual pair
  T* w0; T* w1;        // A z pair
  T* s0; T* s1;        // A p pair
  T* p;                // search direction (read and written by the owner only)
  T* dout;             // damage solve: output array (read at set-up when start = 1)
  T* mte;              // per-solve mass coefficient of each tile element
  T* b; T* dinv;
  uint8_t* W0; uint8_t* W1;   // held-set pair (flipped by restart and check passes)
  double tol;
  int32_t max_iter;
  int32_t kind;        // CG_QP or CG_LINEAR
  int32_t start;       // 1: extrapolated start for the damage solve
  // Chebyshev-Jacobi preconditioner (degree cheb >= 2)
  T* zb;               // z = M r of the current iteration (written by the A z pass)
  T* y0; T* y1;        // Chebyshev iterate pair
  T* dv;               // Chebyshev update direction (owner only)
  int32_t cheb;        // polynomial degree
  int32_t stage;       // pass within a round: 0 main pass, 1 .. cheb-2 Chebyshev steps, cheb-1 the A z pass
  // combination of the round in the pass's last workgroup (Jacobi rounds):
  // 0 none (a k_dmg_red launch follows), 1 combine and advance the solver,
  // 2 combine and run the state machine without storing it (timing aid)
  int32_t fuse;
  uint32_t* arrive;    // arrival counters (see kArriveGroup)
  int32_t nch;         // element chunks of a pass (1, 2): the corner-value space holds 3 / nch values per element
};

// Chebyshev-Jacobi preconditioner z = p(D^-1 A) D^-1 r: `cheb` steps of the
// Chebyshev iteration for A y = r from y = 0 with Jacobi scaling on the
// interval [lmax/kChebRatio, lmax] (Saad, Iterative Methods for Sparse Linear
// Systems, Sec. 12.3): with theta, delta the centre and half-width of the
// interval, sigma = theta/delta, rho_0 = 1/sigma,
//   y_1 = D^-1 r / theta,  d_0 = y_1,
//   rho_j = 1/(2 sigma - rho_{j-1}),
//   d_j = rho_j rho_{j-1} d_{j-1} + (2 rho_j/delta) D^-1 (r - A y_j),  y_{j+1} = y_j + d_j.
// Every eigenvalue of D^-1 A lies in (0, lmax] (lmax a Gershgorin bound), where
// the polynomial is positive, so M is symmetric positive definite and CG
// applies unchanged.
constexpr double kChebRatio = 10.0;

struct ChebCoef {
  double inv_theta, c1, c2;   // 1/theta; c1, c2 of step j: d_j = c1 d_{j-1} + c2 D^-1 res
};

__device__ __forceinline__ ChebCoef cheb_coef(double lmax, int j) {
  const double b = fmax(lmax, 1.0), a = b / kChebRatio;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
  double rp = 1.0 / sigma, rj = rp;
  for (int i = 1; i <= j; ++i) {
    rp = rj;
    rj = 1.0 / (2.0 * sigma - rp);
  }
  ChebCoef c;
  c.inv_theta = 1.0 / theta;
  c.c1 = rj * rp;
  c.c2 = 2.0 * rj / delta;
  return c;
}

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
  c.wbuf = 0;
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

template <typename T, int NPT, bool CHEB, bool FUSE, int NCH>
__global__ __launch_bounds__(kBlock) void k_dmg(DmgArgs<T> a) {
  __shared__ double red[8 * 4 * kWaves];
  const int tile = tile_of_block(a.dm.n_tiles);
  const TileRec t = a.dm.tiles[tile];
  const Ctl* c = a.ctl + t.inst;
  const int mode = c->mode;
  if (mode == MODE_DONE) return;
  // the corner lists do not depend on the solver state: their loads go
  // first, once a finished solve's pass has left
  StagedCorners<2, 12> scn;   // 256 threads: 512 offsets, 3072 corner ids in registers
  stage_corners_load(a.dm, t, scn);
  // Chebyshev steps and the A z pass follow the main pass of first / iterate rounds only
  const int stage = CHEB ? a.stage : 0;
  if (CHEB && stage > 0 && (mode == MODE_RESTART || mode == MODE_CHECK)) return;
  const InstP<T> P = a.ip[t.inst];
  const bool qp = (a.kind == CG_QP);
  const bool projected = qp && (P.bounds == PF_BOUNDS_PROJECTED);
  const bool monotone = projected && (c->flavor != 0);
  const bool xpass = (mode == MODE_RESTART || mode == MODE_CHECK);
  const bool iter = (mode == MODE_ITER);
  const bool setup = xpass && (c->setup != 0);
  const bool cut = xpass && (c->hit != 0);
  const bool release = c->release != 0;
  const bool cur1 = c->pbuf != 0;
  const double alpha = c->alpha, beta = c->beta, amax = c->amax;
  const T al = T(alpha), be = T(beta);
  const double tol = a.tol;
  // current halves (read) and next halves (written) of the pairs
  const T* __restrict__ xc = cur1 ? a.x1 : a.x0;
  const T* __restrict__ rc = cur1 ? a.r1 : a.r0;
  const T* __restrict__ wc = cur1 ? a.w1 : a.w0;
  const T* __restrict__ sc = cur1 ? a.s1 : a.s0;
  T* xn_ = cur1 ? a.x0 : a.x1;
  T* rn_ = cur1 ? a.r0 : a.r1;
  T* wn_ = cur1 ? a.w0 : a.w1;
  T* sn_ = cur1 ? a.s0 : a.s1;
  const bool wcur1 = c->wbuf != 0;
  const uint8_t* __restrict__ Wc = wcur1 ? a.W1 : a.W0;
  uint8_t* Wn = wcur1 ? a.W0 : a.W1;

  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  T* sv = reinterpret_cast<T*>(smem);          // [nloc] the vector the pass multiplies by A
  // after sv (8-byte aligned): iteration passes keep the element corner values
  // of A^e z^e in T; restart and check passes keep them in FP64 (the true
  // residual is then accurate to the rounding of x, not of an FP32 matvec) a
  // chunk of elements at a time; the set-up sweep keeps those FP64 values
  // beside its diagonal corners and loads
  uint16_t* coffs = reinterpret_cast<uint16_t*>(sv + nloc);   // [n_own + 1] corner-list offsets
  uint16_t* clist = coffs + t.n_own + 1;                     // [n_corner] corner ids
  unsigned char* rest =
      smem + ((size_t(nloc) * sizeof(T) + 2 * (size_t(t.n_own) + 1 + size_t(t.n_corner)) + 7) & ~size_t(7));
  T* qc = reinterpret_cast<T*>(rest);          // [3 n_telem] (first, iterate)
  double* qd = reinterpret_cast<double*>(rest); // [3 chunk]   (restart, check)
  const int tid = threadIdx.x;


  // Chebyshev coefficients of this pass's step (the main pass makes step 1)
  ChebCoef chc{1.0, 0.0, 0.0};
  if (CHEB) chc = cheb_coef(c->lmax, stage + 1);
  const T ith = T(chc.inv_theta);
  const T* __restrict__ ysrc = ((stage - 1) & 1) ? a.y1 : a.y0;   // y_j read by stage j-1 >= 1

  // ---- phase 1: the vector to multiply, on owned and halo nodes -------------
  double amin = INFINITY, ch = 0.0;
  // first / iterate main passes: every owned-node load is issued before any
  // update, and r, D^-1 and the held flag stay in registers for phase 3
  const bool fast = !xpass && stage == 0;
  T rz_r[NPT], di_r[NPT];
  uint8_t wf_r[NPT];
  if (fast) {
    T rv_r[NPT], wc_r[NPT], sc_r[NPT], p_r[NPT], x_r[NPT], zb_r[NPT], lb_r[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      const int g = t.node_begin + min(i, t.n_own - 1);
      wf_r[r] = Wc[g];
      di_r[r] = a.dinv[g];
      rv_r[r] = rc[g];
      if (iter) {
        wc_r[r] = wc[g];
        sc_r[r] = (beta == 0.0) ? T(0) : sc[g];
        p_r[r] = (beta == 0.0) ? T(0) : a.p[g];
        x_r[r] = xc[g];
        zb_r[r] = CHEB ? a.zb[g] : T(0);
        lb_r[r] = projected ? a.lb[g] : T(0);
      }
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      if (i >= t.n_own) continue;
      const int g = t.node_begin + i;
      const uint8_t wf = wf_r[r];
      const T di = di_r[r];
      const T rv = rv_r[r];
      T v;
      if (!iter) {
        v = wf ? T(0) : (CHEB ? di * rv * ith : di * rv);
        rz_r[r] = rv;
      } else {
        const T sn = (beta == 0.0) ? wc_r[r] : wc_r[r] + be * sc_r[r];
        const T rn = rv - al * sn;
        v = wf ? T(0) : (CHEB ? di * rn * ith : di * rn);
        const T zv = wf ? T(0) : (CHEB ? zb_r[r] : di * rv);
        const T pv = (beta == 0.0) ? zv : zv + be * p_r[r];
        const T xv = x_r[r];
        T xn = xv + al * pv;
        if (monotone && !wf) {
          const double lbv = double(lb_r[r]);
          if (pv < T(0)) amin = fmin(amin, (lbv - double(xv)) / double(pv));
          if (pv > T(0)) amin = fmin(amin, (1.0 - double(xv)) / double(pv));
          xn = clamp01<T>(xn, T(lbv));
        } else if (projected && !wf) {
          const double xd = double(xn);
          if (double(lb_r[r]) - xd > tol || xd - 1.0 > tol) ch += 1.0;
        }
        a.p[g] = pv;
        sn_[g] = sn;
        xn_[g] = xn;
        rn_[g] = rn;
        rz_r[r] = rn;
      }
      sv[i] = v;
    }
  }
  for (int i = fast ? t.n_own + tid : tid; i < nloc; i += kBlock) {
    const bool own = i < t.n_own;
    const int g = own ? t.node_begin + i : a.dm.halo_idx[t.halo_begin + (i - t.n_own)];
    T v;
    if (CHEB && stage > 0) {
      v = ysrc[g];   // the Chebyshev iterate of the previous pass (0 on held nodes)
    } else if (setup && qp) {
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
    } else if (xpass) {
      v = xc[g];
      if (cut && Wc[g] == HELD_NONE) {
        // monotone flavour: the last step cut at the first bound (step amax
        // along p, whose A p is in the other half of the s pair), then a
        // projected Jacobi-gradient step
        const T am = T(amax);
        const T xh = v + am * a.p[g];
        const T rh = rc[g] - am * sn_[g];
        v = clamp01<T>(xh + T(kExpandStep) * a.dinv[g] * rh, a.lb[g]);
      }
    } else if (!iter) {
      // first pass of a CG run: z = M r (Jacobi), or y_1 = D^-1 r / theta (Chebyshev)
      v = Wc[g] ? T(0) : (CHEB ? a.dinv[g] * rc[g] * ith : a.dinv[g] * rc[g]);
    } else {
      const uint8_t wf = Wc[g];
      const T di = a.dinv[g];
      const T rv = rc[g];
      const T sn = (beta == 0.0) ? wc[g] : wc[g] + be * sc[g];   // s = A p of this iteration
      const T rn = rv - al * sn;
      // z of the next iteration (Jacobi), or the first Chebyshev iterate y_1
      v = wf ? T(0) : (CHEB ? di * rn * ith : di * rn);
      if (own) {
        const T zv = wf ? T(0) : (CHEB ? a.zb[g] : di * rv);
        const T pv = (beta == 0.0) ? zv : zv + be * a.p[g];
        const T xv = xc[g];
        T xn = xv + al * pv;
        if (monotone && !wf) {
          // largest step that keeps this node inside [d_prev, 1]
          const double lbv = double(a.lb[g]);
          if (pv < T(0)) amin = fmin(amin, (lbv - double(xv)) / double(pv));
          if (pv > T(0)) amin = fmin(amin, (1.0 - double(xv)) / double(pv));
          xn = clamp01<T>(xn, T(lbv));
        } else if (projected && !wf) {
          const double xd = double(xn);
          if (double(a.lb[g]) - xd > tol || xd - 1.0 > tol) ch += 1.0;   // free node outside the bounds
        }
        a.p[g] = pv;
        sn_[g] = sn;
        xn_[g] = xn;
        rn_[g] = rn;
      }
    }
    sv[i] = v;
  }
  stage_corners_store(a.dm, t, scn, coffs, clist);

  // ---- set-up: load vector, Jacobi diagonal, per-solve mass coefficients ----
  // The space after sv holds the corner values of one pass; restart and check
  // passes (FP64 values) and the set-up sweep work through the tile's
  // elements in chunks that fit it, each owned node adding the corners of a
  // chunk in its fixed corner order.
  const T* __restrict__ geo = static_cast<const T*>(a.dm.geo);
  const size_t nte = size_t(a.dm.n_te);
  // per-element toughness factor phi_e (Gc_e = Gc phi_e) scales every Gc
  // term of the element's operator and load; absent, phi_e = 1 exactly
  const T* __restrict__ gcs = static_cast<const T*>(a.dm.gcs);
  // the element operator is kap phi_e K^e + mA (1 + delta_kl) with K^e given by
  // its off-diagonals K01, K02, K12 (rows of K^e sum to zero), so a pass reads
  // three values per element instead of the six gradients and the area:
  //   (A^e z)_k = kap phi_e sum_{l != k} K_kl (z_l - z_k) + mA (z_k + z_0 + z_1 + z_2)
  const T* __restrict__ kw = static_cast<const T*>(a.dm.kw);
  // restart / check: FP64 sums of each owned node's corner values of A x
  constexpr bool kFusedSetup = sizeof(T) == 8;   // the set-up sweep sums them too
  double qacc[NPT];
  // set-up: b and D^-1 of the owned nodes, kept for the true residual
  T bset[NPT], dset[NPT];
  if (setup) {
    T dacc[NPT], bacc[NPT], sacc[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) dacc[r] = T(0), bacc[r] = T(0), sacc[r] = T(0), qacc[r] = 0.0;
    // One sweep over the tile's elements assembles the load, the diagonal and
    // the mass coefficients and, in FP64, takes the FP64 corner values of A x
    // with the same element operator (FP32 tiles take them in the restart
    // sweep below, which measured faster there): per element 4 values of
    // width w (7 with the Chebyshev preconditioner's absolute row sums), plus
    // 3 doubles in FP64, as many elements per chunk as the corner space holds
    // (chunks split each node's corner sequence without reordering it, so no
    // sum depends on the chunking).
    constexpr int eb = (kFusedSetup ? 3 * int(sizeof(double)) : 0) + (CHEB ? 7 : 4) * int(sizeof(T));
    const int space = 3 * int(sizeof(T)) * (NCH == 1 ? t.n_telem : (t.n_telem + 1) / 2);
    const int chs = max(1, space / eb);
    double* qs = reinterpret_cast<double*>(rest);   // [3 chunk] FP64 corner values of A x (FP64 tiles)
    T* dcs = reinterpret_cast<T*>(qs + (kFusedSetup ? 3 * chs : 0));   // [3 chunk] diagonal corners
    T* bcs = dcs + 3 * chs;                         // [chunk]   load per corner
    T* scs = bcs + chs;                             // [3 chunk] absolute row sums per corner (Chebyshev)
    for (int e0 = 0; e0 < t.n_telem; e0 += chs) {
      const int e1 = min(e0 + chs, t.n_telem);
      __syncthreads();
      for (int e = e0 + tid; e < e1; e += kBlock) {
        const int te = t.telem_begin + e;
        const T A = geo[6 * nte + te];
        const T w01 = kw[te], w02 = kw[nte + te], w12 = kw[2 * nte + te];
        const T ph = gcs ? gcs[te] : T(1);
        const T kp = P.kap * ph;
        const T He = a.H[a.dm.te_gid[te]];
        const T mA = (P.c0 * ph + P.cH * He) * A * T(1.0 / 12.0);
        a.mte[te] = mA;
        const int l = e - e0;
        // diagonal of K^e from the zero row sums
        dcs[3 * l + 0] = kp * -(w01 + w02) + T(2) * mA;
        dcs[3 * l + 1] = kp * -(w01 + w12) + T(2) * mA;
        dcs[3 * l + 2] = kp * -(w02 + w12) + T(2) * mA;
        bcs[l] = qp ? (P.b0 * ph + P.bH * He) * A * T(1.0 / 3.0) : T(0);
        if (CHEB) {
          // off-diagonal entries of the element matrix
          const T o01 = fabs(kp * w01 + mA);
          const T o02 = fabs(kp * w02 + mA);
          const T o12 = fabs(kp * w12 + mA);
          scs[3 * l + 0] = dcs[3 * l + 0] + o01 + o02;
          scs[3 * l + 1] = dcs[3 * l + 1] + o01 + o12;
          scs[3 * l + 2] = dcs[3 * l + 2] + o02 + o12;
        }
        if constexpr (kFusedSetup) {
          const int c0 = a.dm.lc0[te], c1 = a.dm.lc1[te], c2 = a.dm.lc2[te];
          const double k = double(kp), mm = double(mA);
          const double d01 = w01, d02 = w02, d12 = w12;
          const double s0 = sv[c0], s1 = sv[c1], s2 = sv[c2];
          const double ss = s0 + s1 + s2;
          qs[3 * l + 0] = k * (d01 * (s1 - s0) + d02 * (s2 - s0)) + mm * (s0 + ss);
          qs[3 * l + 1] = k * (d01 * (s0 - s1) + d12 * (s2 - s1)) + mm * (s1 + ss);
          qs[3 * l + 2] = k * (d02 * (s0 - s2) + d12 * (s1 - s2)) + mm * (s2 + ss);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NPT; ++r) {
        const int i = tid + r * kBlock;
        if (i < t.n_own) {
          const int j0 = coffs[i], j1 = coffs[i + 1];
          for (int j = j0; j < j1; ++j) {
            const int cc = clist[j];
            const int e = cc / 3;
            if (e >= e0 && e < e1) {
              dacc[r] += dcs[cc - 3 * e0];
              bacc[r] += bcs[e - e0];
              if (CHEB) sacc[r] += scs[cc - 3 * e0];
              if constexpr (kFusedSetup) qacc[r] += qs[cc - 3 * e0];
            }
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      if (i < t.n_own) {
        const int g = t.node_begin + i;
        if (qp) a.b[g] = bacc[r];
        bset[r] = bacc[r];
        dset[r] = T(1) / dacc[r];
        a.dinv[g] = dset[r];
        // Gershgorin bound of D^-1 A, carried to the reduction as -max in the
        // min-combined slot (unused by restart passes)
        if (CHEB) amin = fmin(amin, -double(sacc[r]) / double(dacc[r]));
      }
    }
  }

  // partials: gamma = r'z, delta = z'Az, max free |r|/A_ii, max held "wants
  // to leave" r/A_ii, held count, max |b|/A_ii (linear set-up), changes
  double gam = 0.0, del = 0.0, cf = 0.0, ca = -INFINITY, na = 0.0, rb = 0.0;
  if (xpass) {
    // ---- restart / check: true residual b - A x with FP64 corner values ----
    // (in FP64 the set-up sweep above has already summed them)
    // FP64 corner values: 2 nch chunks in FP32 (3 doubles per element in the
    // space of 6 floats), nch in FP64
    const int nxc = (sizeof(T) == 4 ? 2 : 1) * NCH;
    const int chx = (t.n_telem + nxc - 1) / nxc;
    const bool summed = kFusedSetup && setup;
    if (!summed) {
#pragma unroll
      for (int r = 0; r < NPT; ++r) qacc[r] = 0.0;
    }
    for (int e0 = 0; !summed && e0 < t.n_telem; e0 += chx) {
      const int e1 = min(e0 + chx, t.n_telem);
      __syncthreads();
      for (int e = e0 + tid; e < e1; e += kBlock) {
        const int te = t.telem_begin + e;
        const int c0 = a.dm.lc0[te], c1 = a.dm.lc1[te], c2 = a.dm.lc2[te];
        const double w01 = kw[te], w02 = kw[nte + te], w12 = kw[2 * nte + te];
        const double k = double(P.kap * (gcs ? gcs[te] : T(1))), mm = double(a.mte[te]);
        const double s0 = sv[c0], s1 = sv[c1], s2 = sv[c2];
        const double ss = s0 + s1 + s2;
        const int l = e - e0;
        qd[3 * l + 0] = k * (w01 * (s1 - s0) + w02 * (s2 - s0)) + mm * (s0 + ss);
        qd[3 * l + 1] = k * (w01 * (s0 - s1) + w12 * (s2 - s1)) + mm * (s1 + ss);
        qd[3 * l + 2] = k * (w02 * (s0 - s2) + w12 * (s1 - s2)) + mm * (s2 + ss);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NPT; ++r) {
        const int i = tid + r * kBlock;
        if (i < t.n_own) {
          const int j0 = coffs[i], j1 = coffs[i + 1];
          for (int j = j0; j < j1; ++j) {
            const int cc = clist[j];
            const int e = cc / 3;
            if (e >= e0 && e < e1) qacc[r] += qd[cc - 3 * e0];
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      if (i >= t.n_own) continue;
      const int g = t.node_begin + i;
      // linear solves read the caller's right-hand side
      const T bi = (summed && qp) ? bset[r] : a.b[g];
      const T ri = T(double(bi) - qacc[r]);
      const T di = summed ? dset[r] : a.dinv[g];
      const double sr = double(ri) * double(di);
      T xv = sv[i];
      uint8_t w = HELD_NONE;
      if (!qp) {
        w = Wc[g];
        if (setup && w == HELD_NONE) rb = fmax(rb, fabs(double(bi) * double(di)));
      } else if (projected) {
        const T lbv = a.lb[g];
        const uint8_t wold = Wc[g];
        if (lbv >= T(1)) {
          w = HELD_FIXED;   // d_prev = 1: the node is fixed
        } else if (mode == MODE_CHECK) {
          const bool viol_lo = wold == HELD_NONE && double(lbv) - double(xv) > tol;
          const bool viol_up = wold == HELD_NONE && double(xv) - 1.0 > tol;
          const bool rel = (wold == HELD_LOWER && sr > kRelease * tol) || (wold == HELD_UPPER && sr < -kRelease * tol);
          w = viol_lo ? HELD_LOWER : (viol_up ? HELD_UPPER : (rel ? HELD_NONE : wold));
          if (viol_lo) xv = lbv;
          if (viol_up) xv = T(1);
          ch += (viol_lo || viol_up || rel) ? 1.0 : 0.0;
        } else if (setup) {
          const uint8_t gs = a.guess ? a.guess[g] : uint8_t(0);
          w = ((gs & PF_ACTIVE_LOWER) && xv <= lbv) ? HELD_LOWER
                                                    : (((gs & PF_ACTIVE_UPPER) && xv >= T(1)) ? HELD_UPPER : HELD_NONE);
        } else if (!monotone) {
          w = wold;
        } else {
          const bool want_lo = ri < T(0) || (wold == HELD_LOWER && !(release && sr > kRelease * tol));
          const bool want_up = ri > T(0) || (wold == HELD_UPPER && !(release && sr < -kRelease * tol));
          w = (xv <= lbv && want_lo) ? HELD_LOWER : ((xv >= T(1) && want_up) ? HELD_UPPER : HELD_NONE);
        }
        if (mode == MODE_RESTART && !monotone && w != HELD_FIXED) {
          // what a check pass of this state would change: it would see the
          // same x, held set and residual, so a restart whose free residual
          // passes and which counts nothing here ends the solve itself
          const bool viol = w == HELD_NONE && (double(lbv) - double(xv) > tol || double(xv) - 1.0 > tol);
          const bool rel = (w == HELD_LOWER && sr > kRelease * tol) || (w == HELD_UPPER && sr < -kRelease * tol);
          ch += (viol || rel) ? 1.0 : 0.0;
        }
      }
      xn_[g] = xv;
      rn_[g] = ri;
      Wn[g] = w;
      if (w) {
        if (w != HELD_FIXED) ca = fmax(ca, w == HELD_UPPER ? -sr : sr);
        na += 1.0;
      } else {
        cf = fmax(cf, fabs(sr));
      }
    }
  } else {
    // ---- first / iterate: corner values of A^e z^e in T ----------------------
    // NCH chunks of the tile's elements; each owned node adds the chunk's
    // entries of its corner list (ascending) from where the previous chunk
    // stopped, so every node's sum runs in the same order for any NCH
    T qacc[NPT];
    int jc[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) qacc[r] = T(0);
    const int che = NCH == 1 ? t.n_telem : (t.n_telem + NCH - 1) / NCH;
#pragma unroll 1
    for (int e0 = 0; e0 < t.n_telem; e0 += che) {
      const int e1 = min(e0 + che, t.n_telem);
      __syncthreads();
      for (int e = e0 + tid; e < e1; e += kBlock) {
        const int te = t.telem_begin + e;
        const int c0 = a.dm.lc0[te], c1 = a.dm.lc1[te], c2 = a.dm.lc2[te];
        const T w01 = kw[te], w02 = kw[nte + te], w12 = kw[2 * nte + te];
        const T kp = P.kap * (gcs ? gcs[te] : T(1));
        const T mA = a.mte[te];
        const T s0 = sv[c0], s1 = sv[c1], s2 = sv[c2];
        const T ss = s0 + s1 + s2;
        const int l = e - e0;
        qc[3 * l + 0] = kp * (w01 * (s1 - s0) + w02 * (s2 - s0)) + mA * (s0 + ss);
        qc[3 * l + 1] = kp * (w01 * (s0 - s1) + w12 * (s2 - s1)) + mA * (s1 + ss);
        qc[3 * l + 2] = kp * (w02 * (s0 - s2) + w12 * (s1 - s2)) + mA * (s2 + ss);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NPT; ++r) {
        const int i = tid + r * kBlock;
        if (i >= t.n_own) continue;
        const int j1 = coffs[i + 1];
        if constexpr (NCH == 1) {
          T q = T(0);
          for (int j = coffs[i]; j < j1; ++j) q += qc[clist[j]];
          qacc[r] = q;
        } else {
          const int cend = 3 * e1, cbeg = 3 * e0;
          int j = (e0 == 0) ? int(coffs[i]) : jc[r];
          T q = qacc[r];
          for (; j < j1; ++j) {
            const int cc = clist[j];
            if (cc >= cend) break;
            q += qc[cc - cbeg];
          }
          qacc[r] = q;
          jc[r] = j;
        }
      }
    }
    T* wn = iter ? wn_ : (cur1 ? a.w1 : a.w0);
    const T* rz = iter ? rn_ : rc;
    T* ydst = (stage & 1) ? a.y1 : a.y0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int i = tid + r * kBlock;
      if (i >= t.n_own) continue;
      const int g = t.node_begin + i;
      const T qi = qacc[r];
      if (CHEB && stage < a.cheb - 1) {
        // Chebyshev step stage + 1: qi = A y_j; d_j and y_{j+1} = y_j + d_j (0 on held nodes)
        const uint8_t w = fast ? wf_r[r] : Wc[g];
        const T rv = fast ? rz_r[r] : rz[g];
        const T yv = sv[i];
        const T res = (fast ? di_r[r] : a.dinv[g]) * (rv - qi);
        const T dj = w ? T(0) : T(chc.c1) * (stage == 0 ? yv : a.dv[g]) + T(chc.c2) * res;
        ydst[g] = w ? T(0) : yv + dj;
        a.dv[g] = dj;
        if (stage == 0) {
          const double sr = double(rv) * double(di_r[r]);
          if (w) {
            if (w != HELD_FIXED) ca = fmax(ca, w == HELD_UPPER ? -sr : sr);
          } else {
            cf = fmax(cf, fabs(sr));
          }
        }
        continue;
      }
      wn[g] = qi;
      if (CHEB) {
        // the A z pass: z = y_cheb, w = A z; the stopping partials came from the main pass
        const T zv = sv[i];
        const T rv = rz[g];   // a later pass of the round: r is read back
        a.zb[g] = zv;
        gam += double(rv) * double(zv);
        del += double(zv) * double(qi);
        continue;
      }
      const T zv = sv[i];
      const T rv = rz_r[r];   // non-Chebyshev first / iterate passes are main passes
      gam += double(rv) * double(zv);
      del += double(zv) * double(qi);
      const double sr = double(rv) * double(di_r[r]);
      const uint8_t w = wf_r[r];
      if (w) {
        if (w != HELD_FIXED) ca = fmax(ca, w == HELD_UPPER ? -sr : sr);
      } else {
        cf = fmax(cf, fabs(sr));
      }
    }
  }
  // with the Chebyshev preconditioner the main pass of a first / iterate
  // round stores every partial but gamma and delta, the A z pass only those
  // two, and the Chebyshev steps none
  uint32_t store = 0xffu;
  if (CHEB && !xpass) {
    if (stage > 0 && stage < a.cheb - 1) return;
    const uint32_t gd = (1u << PT_GAMMA) | (1u << PT_DELTA);
    store = (stage == 0) ? (0xffu & ~gd) : gd;
  }
  double v[8] = {del, amin, gam, cf, ca, na, rb, ch};   // in PT_* order
  const double tot = block_reduce_rows<8, kPartOps>(v, red);
  // partials are stored value-major, [8][n_tiles], so the reduction reads them
  // coalesced; thread k holds value k.  FUSE (Jacobi rounds): stored through
  // to the device-coherent level for the combination in this kernel's last
  // workgroup.
  if constexpr (FUSE) {
    if (tid < 8)
      __hip_atomic_store(&a.part[size_t(tid) * a.dm.n_tiles + tile], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    arrive_and_advance(a, a.ctl + t.inst, tile, P.bounds, red);
  } else {
    if (tid < 8 && (store & (1u << tid))) a.part[size_t(tid) * a.dm.n_tiles + tile] = tot;
  }
}

// Combination of an instance's per-tile partials, in a fixed order: thread t
// adds the partials of tiles tile0 + t, tile0 + t + block, ... in that order,
// then the block's values are reduced (DPP rows, then a fixed-order combine);
// thread k < 8 returns value k.  k_dmg_red runs the same order with the loads
// of kRedBatch tiles per thread in flight (it is latency-bound: one
// workgroup, a few kilobytes; tiles past the end combine as the identity of
// each operation through selects, not a branch, so the loads stay ahead of
// every use).  This flavour, for the last workgroup of a pass, reads one
// tile's partials per thread at a time past this die's L2 (the partials of the
// running kernel) and keeps the pass's register count.
constexpr int kRedBatch = 8;
constexpr int kFuseMaxTiles = 512;   // instances combined in the pass's last workgroup (see run_solve)
__device__ __forceinline__ double combine_partials(double* part, size_t nt, int tile0, int ntiles, double* red) {
  const int tile_end = tile0 + ntiles;
  double v[8] = {0.0, INFINITY, 0.0, 0.0, -INFINITY, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int k = tile0 + int(threadIdx.x); k < tile_end; k += kBlock) {
    double q[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) q[f] = __hip_atomic_load(part + size_t(f) * nt + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v[PT_DELTA] += q[PT_DELTA];
    v[PT_AMIN] = fmin(v[PT_AMIN], q[PT_AMIN]);
    v[PT_GAMMA] += q[PT_GAMMA];
    v[PT_CF] = fmax(v[PT_CF], q[PT_CF]);
    v[PT_CA] = fmax(v[PT_CA], q[PT_CA]);
    v[PT_NA] += q[PT_NA];
    v[PT_RB] = fmax(v[PT_RB], q[PT_RB]);
    v[PT_CH] += q[PT_CH];
  }
  return block_reduce_rows<8, kPartOps>(v, red);
}

// The solver's state machine: one round's combined partials advance the
// instance's control block c (a register copy; the caller stores it).
__device__ __forceinline__ void advance_solver(Ctl* c, const double (&v)[8], int bnd, int kind, double tol,
                                               int max_iter) {
  const int mode = c->mode;
  const double sdel = v[PT_DELTA], samin = v[PT_AMIN], sgam = v[PT_GAMMA], scf = v[PT_CF], sca = v[PT_CA];
  const double sna = v[PT_NA], srb = v[PT_RB], sch = v[PT_CH];
  const bool qp = (kind == CG_QP);
  const bool projected = qp && (bnd == PF_BOUNDS_PROJECTED);
  const bool monotone = projected && (c->flavor != 0);
  const bool setup = c->setup != 0;
  c->iters += 1;
  c->inner = (mode == MODE_ITER) ? c->inner + 1 : 0;
  if (setup && !qp) c->ref = srb;   // linear solves stop relative to max |b_i|/A_ii
  if (setup) c->lmax = (samin < 0.0) ? -samin : 0.0;   // Gershgorin bound of D^-1 A (Chebyshev only)
  const double tl = tol * c->ref;
  const double rs = c->ref > 0.0 ? c->ref : 1.0;
  if (mode == MODE_RESTART || mode == MODE_CHECK) {
    // the pass wrote x, r and the held set into the other halves of their pairs
    c->pbuf ^= 1;
    c->wbuf ^= 1;
    c->setup = 0;
    c->hit = 0;
    c->nact = int32_t(sna);
    c->resid = (monotone ? fmax(scf, sca) : scf) / rs;
    if (!isfinite(scf)) {
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
        c->mode = MODE_FIRST;
      }
    } else if (monotone) {
      if (scf <= tl && sca <= kRelease * tl) {
        c->mode = MODE_DONE;
      } else if (scf <= tl) {
        c->mode = MODE_RESTART;   // face converged, held nodes want to leave: release them
        c->release = 1;
        c->restarts += 1;
      } else {
        c->mode = MODE_FIRST;
      }
    } else if (scf <= tl) {
      // a restart counts the changes a check of its state would make
      c->mode = (projected && sch > 0.0) ? MODE_CHECK : MODE_DONE;
    } else {
      c->mode = MODE_FIRST;
    }
  } else if (mode == MODE_FIRST) {
    if (!isfinite(sgam) || !isfinite(sdel)) {
      c->flags |= PF_FLAG_NONFINITE;
      c->mode = MODE_DONE;
    } else if (!(sdel > 0.0)) {
      // z = 0 on every free node: the free residual vanishes
      c->mode = projected && !monotone ? MODE_CHECK : MODE_RESTART;
      c->release = monotone ? 1 : 0;
    } else {
      c->alpha = sgam / sdel;
      c->beta = 0.0;
      c->rz = sgam;
      c->mode = MODE_ITER;
    }
  } else if (monotone && samin < c->alpha) {
    // the step crosses a bound: cut it there and restart (x, r stay in the
    // current halves; p and s = A p of this step are kept for the cut)
    c->amax = fmax(samin, 0.0);
    c->hit = 1;
    c->release = 0;
    c->restarts += 1;
    c->mode = MODE_RESTART;
  } else {
    c->pbuf ^= 1;
    c->resid = scf / rs;
    const double beta = sgam / c->rz;
    const double den = sdel - beta * sgam / c->alpha;
    const bool early = projected && !monotone && c->inner >= 2 && sch > 0.25 * double(c->nnodes - c->nact);
    if (!isfinite(sgam) || !isfinite(sdel)) {
      c->flags |= PF_FLAG_NONFINITE;
      c->mode = MODE_DONE;
    } else if (scf <= tl || sgam == 0.0 || early || !(den > 0.0)) {
      // this CG run converged on its recurrence residual, a quarter of the
      // free nodes already left their bounds, or the recurrence lost
      // definiteness: recompute the true residual (and update the held set)
      if (projected && !monotone) {
        c->mode = MODE_CHECK;
      } else {
        c->mode = MODE_RESTART;
        c->release = (monotone && sca > kRelease * tl) ? 1 : 0;
        c->restarts += monotone ? 1 : 0;
      }
    } else {
      c->beta = beta;
      c->alpha = sgam / den;
      c->rz = sgam;
    }
  }
  if (c->mode != MODE_DONE && c->iters >= max_iter) {
    c->flags |= PF_FLAG_NOT_CONVERGED;
    c->mode = MODE_DONE;
  }
}

// One workgroup per instance: combine the tiles' partials and advance the
// state (the rounds of the Chebyshev-preconditioned solver, and passes run
// without the combination in their last workgroup).
constexpr int kRedBlock = kBlock;
__global__ __launch_bounds__(kRedBlock) void k_dmg_red(Ctl* ctl, const double* part, int n_tiles, const int* bounds,
                                                       int kind, double tol, int max_iter) {
  __shared__ double red[8 * 4 * (kRedBlock / 64)];
  __shared__ double tot[8];
  Ctl* const cp = ctl + blockIdx.x;
  Ctl cc;
  int bnd = 0;
  if (threadIdx.x == 0) {
    cc = *cp;
    bnd = bounds[blockIdx.x];
  }
  if (cp->mode == MODE_DONE) return;
  const int tile_end = cp->tile0 + cp->ntiles;
  double v[8] = {0.0, INFINITY, 0.0, 0.0, -INFINITY, 0.0, 0.0, 0.0};
  const size_t nt = size_t(n_tiles);
#pragma unroll 1
  for (int k0 = cp->tile0 + threadIdx.x; k0 < tile_end; k0 += kRedBatch * kRedBlock) {
    double q[kRedBatch][8];
#pragma unroll
    for (int j = 0; j < kRedBatch; ++j) {
      const int k = min(k0 + j * kRedBlock, tile_end - 1);   // clamped: loaded, not added
#pragma unroll
      for (int f = 0; f < 8; ++f) q[j][f] = part[size_t(f) * nt + k];
    }
#pragma unroll
    for (int j = 0; j < kRedBatch; ++j) {
      const bool in = k0 + j * kRedBlock < tile_end;
      v[PT_DELTA] += in ? q[j][PT_DELTA] : 0.0;
      v[PT_AMIN] = fmin(v[PT_AMIN], in ? q[j][PT_AMIN] : INFINITY);
      v[PT_GAMMA] += in ? q[j][PT_GAMMA] : 0.0;
      v[PT_CF] = fmax(v[PT_CF], in ? q[j][PT_CF] : -INFINITY);
      v[PT_CA] = fmax(v[PT_CA], in ? q[j][PT_CA] : -INFINITY);
      v[PT_NA] += in ? q[j][PT_NA] : 0.0;
      v[PT_RB] = fmax(v[PT_RB], in ? q[j][PT_RB] : -INFINITY);
      v[PT_CH] += in ? q[j][PT_CH] : 0.0;
    }
  }
  const double vk = block_reduce_rows<8, kPartOps, kRedBlock / 64>(v, red);
  if (threadIdx.x < 8) tot[threadIdx.x] = vk;
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = tot[k];
  advance_solver(&cc, v, bnd, kind, tol, max_iter);
  *cp = cc;
}

// The end of a Jacobi round's pass: each workgroup counts its arrival once its
// partial sums are stored, and the instance's last workgroup to arrive
// combines every tile's partials and advances the solver, so a round is one
// launch.  Nothing waits for anything: a workgroup that is not last exits.
// The partials are stored through to the device-coherent level (the L2s of
// the chip's dies are not coherent with each other) and counted only after
// the stores have completed; the last workgroup reads them past its L2.  The
// fixed combination order is that of k_dmg_red, so the bits are the same.
template <typename T>
__device__ __forceinline__ void arrive_and_advance(const DmgArgs<T>& a, Ctl* c, int tile, int bnd, double* red) {
  __shared__ int s_last;
  __shared__ double s_tot[8];
  const int tid = threadIdx.x;
  uint32_t* const top = a.arrive + size_t(c->cbase + c->ngroup) * kArriveStride;
  if (tid < 64) {
    // threads 0-7 of this wave stored the partials: wait for the stores
    __builtin_amdgcn_s_waitcnt(0);
    if (tid == 0) {
      const int g = (tile - c->tile0) / kArriveGroup;
      const unsigned gsize = unsigned(min(kArriveGroup, c->ntiles - g * kArriveGroup));
      uint32_t* const gc = a.arrive + size_t(c->cbase + g) * kArriveStride;
      bool last = false;
      if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
        __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               unsigned(c->ngroup) - 1;
      }
      s_last = last;
    }
  }
  __syncthreads();
  if (!s_last) return;
  const double vk = combine_partials(a.part, size_t(a.dm.n_tiles), c->tile0, c->ntiles, red);
  if (tid < 8) s_tot[tid] = vk;
  __syncthreads();
  if (tid != 0) return;
  Ctl cc = *c;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = s_tot[k];
  advance_solver(&cc, v, bnd, a.kind, a.tol, a.max_iter);
  if (a.fuse == 1) *c = cc;
  __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Final pass: bounds, active flags and statistics.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dmg_final(DmgArgs<T> a, uint8_t* active_out, pf_cg_stats_t* stats) {
  const int tile = tile_of_block(a.dm.n_tiles);
  const TileRec t = a.dm.tiles[tile];
  const Ctl* c = a.ctl + t.inst;
  const InstP<T> P = a.ip[t.inst];
  const bool projected = (P.bounds == PF_BOUNDS_PROJECTED);
  const T* xc = c->pbuf ? a.x1 : a.x0;
  const uint8_t* Wc = c->wbuf ? a.W1 : a.W0;
  if (a.kind != CG_QP) {
    // the result goes to the caller's array x0
    for (int i = threadIdx.x; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      a.x0[g] = (c->ref == 0.0) ? T(0) : xc[g];
    }
  } else {
    for (int i = threadIdx.x; i < t.n_own; i += kBlock) {
      const int g = t.node_begin + i;
      T xv = xc[g];
      const T lbv = a.lb[g];
      uint8_t act = 0;
      if (projected) {
        const uint8_t w = Wc[g];
        act = (w == HELD_LOWER || w == HELD_FIXED) ? PF_ACTIVE_LOWER : ((w == HELD_UPPER) ? PF_ACTIVE_UPPER : 0);
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
  if (stats && threadIdx.x == 0 && tile == c->tile0) {
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
  // the damage solve iterates in workspaces and writes d at the end; linear
  // solves start from, and end in, the caller's array
  a.x0 = (kind == CG_QP) ? static_cast<T*>(m->dw.xw0) : static_cast<T*>(d);
  a.x1 = static_cast<T*>(m->dw.xw1);
  a.dout = static_cast<T*>(d);
  a.r0 = static_cast<T*>(m->dw.r0);
  a.r1 = static_cast<T*>(m->dw.r1);
  a.w0 = static_cast<T*>(m->dw.w0);
  a.w1 = static_cast<T*>(m->dw.w1);
  a.s0 = static_cast<T*>(m->dw.s0);
  a.s1 = static_cast<T*>(m->dw.s1);
  a.p = static_cast<T*>(m->dw.p);
  a.b = static_cast<T*>(m->dw.b);
  a.dinv = static_cast<T*>(m->dw.dinv);
  a.W0 = m->dw.wset;
  a.W1 = m->dw.wset + m->n_nodes;
  a.tol = tol;
  a.max_iter = max_iter;
  a.zb = a.y0 = a.y1 = a.dv = nullptr;
  a.cheb = 0;
  a.stage = 0;
  a.fuse = 0;
  a.arrive = m->dw.arrive;
  a.nch = 1;
  return a;
}

// The damage pass for npt owned nodes per thread (a tile of up to 256 npt
// owned nodes) with its elements in nch chunks.
template <typename T, int NPT, bool CHEB, bool FUSE>
static void (*dmg_kernel_c(int nch))(DmgArgs<T>) {
  return nch == 2 ? k_dmg<T, NPT, CHEB, FUSE, 2> : k_dmg<T, NPT, CHEB, FUSE, 1>;
}
template <typename T, bool CHEB, bool FUSE>
static void (*dmg_kernel(int npt, int nch))(DmgArgs<T>) {
  return npt <= 1 ? dmg_kernel_c<T, 1, CHEB, FUSE>(nch)
                  : (npt <= 2 ? dmg_kernel_c<T, 2, CHEB, FUSE>(nch)
                              : (npt <= 4 ? dmg_kernel_c<T, 4, CHEB, FUSE>(nch) : dmg_kernel_c<T, 8, CHEB, FUSE>(nch)));
}

// Element chunks of the damage passes: two when halving the corner-value
// space in LDS lets every tile's workgroup be resident at once where one
// chunk cannot (the workgroups per CU from the kernel's registers and LDS).
// A second wave that holds only the tiles the first could not place moves a
// fraction of the pass's bytes but adds most of a pass's latency; with
// several waves either way the second chunk's extra barrier and element
// phase cost more than the shorter tail saves.
template <typename T>
static int damage_chunks(pf_mesh_s* m) {
  if (m->dmg_nch > 0) return m->dmg_nch;
  int nch = m->damage_chunks;
  if (nch <= 0) {
    const int npt = (m->max_own + kBlock - 1) / kBlock;
    const void* k1 = reinterpret_cast<const void*>(dmg_kernel<T, false, false>(npt, 1));
    const void* k2 = reinterpret_cast<const void*>(dmg_kernel<T, false, false>(npt, 2));
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    auto waves = [&](const void* k, size_t lds) -> long {
      int occ = 0;
      if (ncu <= 0 || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kBlock, lds) != hipSuccess || occ <= 0)
        return LONG_MAX;
      const long slots = long(occ) * ncu;
      return (long(m->n_tiles) + slots - 1) / slots;
    };
    nch = (waves(k2, size_t(m->max_lds_damage2)) == 1 && waves(k1, size_t(m->max_lds_damage)) > 1) ? 2 : 1;
  }
  m->dmg_nch = nch;
  return nch;
}

void damage_plan(pf_mesh_s* m) {
  if (m->dtype == PF_F64)
    (void)damage_chunks<double>(m);
  else
    (void)damage_chunks<float>(m);
}

static size_t damage_lds(const pf_mesh_s* m, int nch) {
  return size_t(nch == 2 ? m->max_lds_damage2 : m->max_lds_damage);
}

template <typename T>
static pf_status_t run_solve(pf_mesh_s* m, int kind, const void* H, const void* d_prev, void* d,
                             const uint8_t* guess, uint8_t* active_out, const pf_cg_opts_t* o,
                             pf_cg_stats_t* stats, hipStream_t s) {
  DmgArgs<T> a = dmg_args<T>(m, kind, H, d_prev, d, guess, o->tol, o->max_iter, o->start);
  const dim3 grid(m->n_tiles), block(kBlock), igrid(m->n_inst);
  a.nch = damage_chunks<T>(m);
  const size_t lds = damage_lds(m, a.nch);
  if (!o->resume) {
    timer_begin(m, 2, s);
    hipLaunchKernelGGL(k_dmg_init, dim3((m->n_inst + 63) / 64), dim3(64), 0, s, m->dw.ctl, m->n_inst, kind,
                       o->monotone);
    timer_end(m, 2, s);
  }
  const int npt = (m->max_own + kBlock - 1) / kBlock;
  const bool cheb = o->precond >= 2;
  a.cheb = cheb ? o->precond : 0;
  // Jacobi rounds of instances of up to kFuseMaxTiles tiles combine their
  // partials in the pass's last workgroup (one launch per round: the last
  // workgroup's combination takes one memory round trip per 256 tiles, which
  // beats the separate reduction launch only while there are few); larger
  // instances and Chebyshev rounds keep the reduction launch
  a.fuse = (!cheb && m->max_inst_tiles <= kFuseMaxTiles) ? 1 : 0;
  a.zb = static_cast<T*>(m->dw.zb);
  a.y0 = static_cast<T*>(m->dw.y0);
  a.y1 = static_cast<T*>(m->dw.y1);
  a.dv = static_cast<T*>(m->dw.dv);
  auto kdmg = cheb ? dmg_kernel<T, true, false>(npt, a.nch)
                   : (a.fuse ? dmg_kernel<T, false, true>(npt, a.nch) : dmg_kernel<T, false, false>(npt, a.nch));
  if (kind == CG_QP) {
    const unsigned char* ab = reinterpret_cast<const unsigned char*>(&a);
    m->last_qp_args.assign(ab, ab + sizeof(a));
    m->last_qp_cheb = a.cheb;
  }
  auto round = [&]() {
    // one pass, or with the Chebyshev preconditioner one pass per matrix-vector product
    for (int st = 0; st < (cheb ? a.cheb : 1); ++st) {
      DmgArgs<T> as = a;
      as.stage = st;
      timer_begin(m, 1, s);
      hipLaunchKernelGGL(kdmg, grid, block, lds, s, as);
      timer_end(m, 1, s);
    }
    if (a.fuse) return;
    timer_begin(m, 4, s);
    hipLaunchKernelGGL(k_dmg_red, igrid, dim3(kRedBlock), 0, s, m->dw.ctl, m->dw.part, m->n_tiles, m->dw.bounds,
                       kind, o->tol, o->max_iter);
    timer_end(m, 4, s);
  };
  const int max_rounds = (o->check_every <= 0 && o->rounds > 0) ? std::min(o->rounds, o->max_iter) : o->max_iter;
  int launched = 0;
  if (o->check_every <= 0) {
    for (; launched < max_rounds; ++launched) round();
  } else {
    // first poll after two rounds more than the last solve of this kind
    // needed (solves of consecutive steps take similar counts, and a round of
    // a finished solve costs only two near-empty launches), then every
    // check_every rounds
    const int last = m->last_rounds[kind == CG_QP ? 0 : 1];
    int chunk = last > 0 ? last + 2 : std::min(o->check_every, 8);
    if (o->check_every == 1) chunk = 1;   // poll after every round: no round runs after the solve ends
    while (launched < max_rounds) {
      const int n = std::min(chunk, max_rounds - launched);
      for (int k = 0; k < n; ++k) round();
      launched += n;
      PF_HIP(hipGetLastError());
      PF_HIP(hipMemcpyAsync(m->ctl_pinned, m->dw.ctl, sizeof(Ctl) * m->n_inst, hipMemcpyDeviceToHost, s));
      PF_HIP(hipEventRecord(m->poll_ev, s));
      // spin rather than block: the wait is short and a sleeping host thread
      // wakes up tens of microseconds late
      hipError_t q;
      while ((q = hipEventQuery(m->poll_ev)) == hipErrorNotReady) {
      }
      if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
      bool all_done = true;
      for (int k = 0; k < m->n_inst; ++k) all_done = all_done && (m->ctl_pinned[k].mode == MODE_DONE);
      if (all_done) break;
      chunk = o->check_every;
    }
  }
  timer_begin(m, 2, s);
  hipLaunchKernelGGL(k_dmg_final<T>, grid, block, 0, s, a, active_out, stats);
  timer_end(m, 2, s);
  PF_HIP(hipGetLastError());
  if (o->check_every > 0) {
    // the last poll saw every instance done, or the round budget is spent:
    // either way the control blocks it copied are final
    int flags = 0, rounds = 0;
    for (int k = 0; k < m->n_inst; ++k) {
      flags |= m->ctl_pinned[k].flags;
      if (m->ctl_pinned[k].mode != MODE_DONE) flags |= PF_FLAG_NOT_CONVERGED;
      rounds = std::max(rounds, int(m->ctl_pinned[k].iters));
    }
    m->last_rounds[kind == CG_QP ? 0 : 1] = rounds;
    if (flags & PF_FLAG_NONFINITE) return fail(PF_ERR_NONFINITE, "non-finite value in the damage CG");
    if (flags & PF_FLAG_NOT_CONVERGED) return fail(PF_ERR_NOT_CONVERGED, "damage CG reached max_iter");
  }
  return PF_OK;
}

// n launches of the main pass of the last damage solve's current round, with
// no reduction in between (a throughput measurement; see pf.h).
template <typename T>
static pf_status_t repeat_pass(pf_mesh_s* m, const void* H, const void* d_prev, void* d, int n, hipStream_t s) {
  DmgArgs<T> a;
  if (m->last_qp_args.size() != sizeof(a)) return fail(PF_ERR_ARG, "no damage solve on this handle");
  if (m->last_qp_cheb != 0) return fail(PF_ERR_ARG, "repeated passes need the Jacobi preconditioner");
  std::memcpy(&a, m->last_qp_args.data(), sizeof(a));
  // the caller's arrays as given now; the workspaces are the handle's
  a.H = static_cast<const T*>(H);
  a.lb = static_cast<const T*>(d_prev);
  a.dout = static_cast<T*>(d);
  a.guess = nullptr;
  // where the solver's rounds combine the partials in the pass's last
  // workgroup, each launch does so too but leaves the control block as it is
  a.fuse = a.fuse ? 2 : 0;
  PF_HIP(hipMemcpyAsync(m->ctl_pinned, m->dw.ctl, sizeof(Ctl) * m->n_inst, hipMemcpyDeviceToHost, s));
  PF_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < m->n_inst; ++k)
    if (m->ctl_pinned[k].mode != MODE_ITER)
      return fail(PF_ERR_ARG, "the last damage solve did not stop in a CG iteration");
  const int npt = (m->max_own + kBlock - 1) / kBlock;
  auto kdmg = a.fuse ? dmg_kernel<T, false, true>(npt, a.nch) : dmg_kernel<T, false, false>(npt, a.nch);
  a.stage = 0;
  for (int i = 0; i < n; ++i)
    hipLaunchKernelGGL(kdmg, dim3(m->n_tiles), dim3(kBlock), damage_lds(m, a.nch), s, a);
  PF_HIP(hipGetLastError());
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
  if (opts->rounds < 0) return fail(PF_ERR_ARG, "rounds must be >= 0");
  if (opts->precond < 0 || opts->precond > 4) return fail(PF_ERR_ARG, "precond must be in [0, 4]");
  if (opts->resume && !m->qp_started) return fail(PF_ERR_ARG, "resume without a previous damage solve on this handle");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = upload_params(m, p, nullptr, s)) != PF_OK) return st;
  m->qp_started = true;
  return damage_cg(m, CG_QP, H, d_prev, d, active_guess, active_out, opts, stats, s);
}

extern "C" pf_status_t pf_damage_pass_repeat(pf_mesh_t m, const void* H, const void* d_prev, void* d,
                                             int32_t n_passes, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "mesh is NULL");
  if (!H || !d_prev || !d) return fail(PF_ERR_ARG, "NULL argument");
  if (n_passes < 1) return fail(PF_ERR_ARG, "n_passes must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return (m->dtype == PF_F64) ? repeat_pass<double>(m, H, d_prev, d, n_passes, s)
                              : repeat_pass<float>(m, H, d_prev, d, n_passes, s);
}
