// Tile-size autotuner: builds the tile plan for each candidate size, times
// the explicit step and a damage CG round on the device, and picks the size
// with the smallest weighted time.  A set-up call: it allocates.
#include <algorithm>
#include <cstring>

#include "pf_internal.hpp"

namespace pf {

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct Handle {
  pf_mesh_t m = nullptr;
  ~Handle() {
    if (m) pf_mesh_destroy(m);
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

constexpr int kDefaultCandidates[] = {128, 192, 256, 384, 448, 512, 768, 1024};

// Time `reps` explicit steps and `reps` damage CG rounds of one tile plan.
pf_status_t time_plan(const pf_mesh_desc_t* inst, int32_t n_inst, pf_dtype_t dtype, const pf_params_t* p,
                      int32_t tile_nodes, int32_t reps, hipStream_t s, double* explicit_us, int32_t* explicit_block,
                      int32_t* explicit_chunks, double* round_us) {
  Handle h;
  pf_tile_opts_t to{tile_nodes, 0, 0, 0};
  pf_status_t st = pf_mesh_create(inst, n_inst, dtype, &to, s, &h.m);
  if (st != PF_OK) return st;
  pf_mesh_s* m = h.m;
  const size_t w = (dtype == PF_F64) ? 8 : 4;
  const size_t N = size_t(m->n_nodes), Ne = size_t(m->n_elems);
  // two zero states for the ping-pong of the explicit step
  DevBuf buf;
  const size_t per_state = 7 * N * w + Ne * w;
  PF_HIP(hipMalloc(&buf.p, 2 * per_state));
  PF_HIP(hipMemsetAsync(buf.p, 0, 2 * per_state, s));
  pf_state_t st2[2] = {};
  for (int k = 0; k < 2; ++k) {
    char* b = static_cast<char*>(buf.p) + k * per_state;
    void** f[8] = {&st2[k].ux, &st2[k].uy, &st2[k].vx, &st2[k].vy, &st2[k].ax, &st2[k].ay, &st2[k].d, &st2[k].H};
    for (int j = 0; j < 7; ++j) *f[j] = b + j * N * w;
    *f[7] = b + 7 * N * w;
  }
  std::vector<double> dt(n_inst);
  if ((st = pf_cfl_dt(m, p, 0.5, dt.data())) != PF_OK) return st;
  Events ev;
  PF_HIP(hipEventCreate(&ev.a));
  PF_HIP(hipEventCreate(&ev.b));
  // explicit step, with each workgroup size and element chunk count
  float ms = 0.f;
  *explicit_us = 0.0;
  for (int cfg = 0; cfg < 4; ++cfg) {
    const int bs = (cfg & 1) ? 512 : 256, nch = (cfg & 2) ? 2 : 1;
    m->explicit_block = bs;
    m->explicit_chunks = nch;
    for (int k = 0; k < 2; ++k)
      if ((st = pf_explicit_step(m, p, dt.data(), &st2[k & 1], &st2[(k + 1) & 1], nullptr, s)) != PF_OK) return st;
    PF_HIP(hipEventRecord(ev.a, s));
    for (int k = 0; k < reps; ++k)
      if ((st = pf_explicit_step(m, p, dt.data(), &st2[k & 1], &st2[(k + 1) & 1], nullptr, s)) != PF_OK) return st;
    PF_HIP(hipEventRecord(ev.b, s));
    PF_HIP(hipEventSynchronize(ev.b));
    PF_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    const double us = 1e3 * double(ms) / reps;
    if (*explicit_us == 0.0 || us < *explicit_us) {
      *explicit_us = us;
      *explicit_block = bs;
      *explicit_chunks = nch;
    }
  }
  // damage CG rounds: a linear solve on all nodes with a positive right-hand
  // side (every byte 0x3f is a positive finite value in either width), run
  // for a fixed number of rounds without synchronising
  PF_HIP(hipMemsetAsync(m->dw.b, 0x3f, N * w, s));
  PF_HIP(hipMemsetAsync(m->dw.wset, 0, N, s));
  PF_HIP(hipMemsetAsync(st2[0].d, 0, N * w, s));
  pf_cg_opts_t o{};
  o.tol = 1e-300;
  o.max_iter = 2;
  o.check_every = 0;
  if ((st = damage_cg(m, CG_LINEAR, st2[0].H, nullptr, st2[0].d, nullptr, nullptr, &o, nullptr, s)) != PF_OK)
    return st;
  PF_HIP(hipMemsetAsync(st2[0].d, 0, N * w, s));
  o.max_iter = reps;
  PF_HIP(hipEventRecord(ev.a, s));
  if ((st = damage_cg(m, CG_LINEAR, st2[0].H, nullptr, st2[0].d, nullptr, nullptr, &o, nullptr, s)) != PF_OK)
    return st;
  PF_HIP(hipEventRecord(ev.b, s));
  PF_HIP(hipEventSynchronize(ev.b));
  PF_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  *round_us = 1e3 * double(ms) / reps;
  return PF_OK;
}

}  // namespace
}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_tune_tiles(const pf_mesh_desc_t* inst, int32_t n_instances, pf_dtype_t dtype,
                                     const pf_params_t* p, const pf_tune_opts_t* opts, pf_tune_result_t* out,
                                     pf_stream_t stream) {
  if (!inst || !p || !out) return fail(PF_ERR_ARG, "NULL argument");
  if (n_instances < 1) return fail(PF_ERR_ARG, "n_instances must be >= 1");
  if (dtype != PF_F32 && dtype != PF_F64) return fail(PF_ERR_ARG, "bad dtype");
  std::vector<int32_t> cand;
  int32_t reps = 20;
  double weight = 16.0;
  if (opts) {
    if (opts->n_candidates < 0 || opts->n_candidates > PF_TUNE_MAX) return fail(PF_ERR_ARG, "n_candidates must be in [0, 8]");
    for (int k = 0; k < opts->n_candidates; ++k) {
      const int32_t c = opts->tile_nodes[k];
      if (c < 64 || c > kMaxTileNodes) return fail(PF_ERR_ARG, "candidate tile_nodes must be in [64, 2048]");
      cand.push_back(c);
    }
    if (opts->reps < 0 || opts->reps > 10000) return fail(PF_ERR_ARG, "reps must be in [0, 10000]");
    if (opts->reps > 0) reps = opts->reps;
    if (opts->cg_rounds_per_step > 0) weight = opts->cg_rounds_per_step;
  }
  if (cand.empty()) cand.assign(std::begin(kDefaultCandidates), std::end(kDefaultCandidates));
  std::memset(out, 0, sizeof(*out));
  out->best = 0;
  double best = 0.0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (size_t k = 0; k < cand.size(); ++k) {
    out->tile_nodes[k] = cand[k];
    double te = 0.0, tr = 0.0;
    int32_t eb = 256, ec = 1;
    const pf_status_t st = time_plan(inst, n_instances, dtype, p, cand[k], reps, s, &te, &eb, &ec, &tr);
    out->status[k] = st;
    out->n_tried = int32_t(k + 1);
    if (st == PF_ERR_UNSUPPORTED) continue;   // the plan needs more LDS than a workgroup has
    if (st != PF_OK) return st;               // a real error: pf_last_error() holds its text
    out->explicit_us[k] = te;
    out->explicit_block[k] = eb;
    out->explicit_chunks[k] = ec;
    out->cg_round_us[k] = tr;
    out->score_us[k] = te + weight * tr;
    if (out->best == 0 || out->score_us[k] < best) {
      best = out->score_us[k];
      out->best = cand[k];
      out->best_explicit_block = eb;
      out->best_explicit_chunks = ec;
    }
  }
  if (out->best == 0) return fail(PF_ERR_UNSUPPORTED, "no candidate tile size fits the device's LDS");
  return PF_OK;
}
