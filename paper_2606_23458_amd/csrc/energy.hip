// Energy budget of a state, per instance and per unit thickness (Sec. 3,
// dynamic SENT energy discussion; the energies of Sec. 2.1-2.2):
//   E_kin  = 1/2 sum_i m_i |v_i|^2                      (lumped mass m_i = rho sum A_e/3)
//   E_el   = sum_e A_e (g(d_e) psi+(eps_e) + psi-(eps_e)),   d_e = mean of the element's nodal d
//   E_frac = Gc/(2 l0) d'Md + Gc l0/2 d'Kd               (AT2)
//          = 3 Gc/(8 l0) (int d + l0^2 d'Kd)             (AT1)
// (with a toughness field each element's share takes its own Gc_e)
// psi- comes from the split's stress: every split's psi+- is homogeneous of
// degree 2 in the strain, so psi- = sigma-:eps / 2.
//
// One workgroup per tile: owned nodes give the kinetic term, owned elements
// the elastic and fracture terms (each element once); per-tile FP64 partials
// are combined per instance in a fixed order by a second launch.
#include <mutex>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "split.hpp"

namespace pf {

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_energy(DevMesh dm, const InstP<T>* __restrict__ ip, StateIn<T> st,
                                                   double* part) {
  __shared__ double red[3 * 4 * kWaves];
  const int tile = tile_of_block(dm.n_tiles);
  const TileRec t = dm.tiles[tile];
  const InstP<T> P = ip[t.inst];
  extern __shared__ __align__(16) unsigned char smem[];
  const int nloc = t.n_own + t.n_halo;
  T* sux = reinterpret_cast<T*>(smem);
  T* suy = sux + nloc;
  T* sd = suy + nloc;
  const int tid = threadIdx.x;
  const T* __restrict__ wl = static_cast<const T*>(dm.wlump);
  const double rho = 1.0 / double(P.inv_rho);
  double ek = 0.0, ee = 0.0, ef = 0.0;
  for (int i = tid; i < nloc; i += kBlock) {
    const bool own = i < t.n_own;
    const int g = own ? t.node_begin + i : dm.halo_idx[t.halo_begin + (i - t.n_own)];
    sux[i] = st.ux[g];
    suy[i] = st.uy[g];
    sd[i] = st.d[g];
    if (own) {
      const double vx = st.vx[g], vy = st.vy[g];
      ek += 0.5 * rho * double(wl[g]) * (vx * vx + vy * vy);
    }
  }
  __syncthreads();
  const T* __restrict__ geo = static_cast<const T*>(dm.geo);
  const size_t nte = size_t(dm.n_te);
  const bool at2 = P.model == PF_AT2;
  const T* __restrict__ gcs = static_cast<const T*>(dm.gcs);
  for (int e = tid; e < t.n_own_elem; e += kBlock) {
    const int te = t.telem_begin + t.own_elem_lo + e;
    const int c0 = dm.lc0[te], c1 = dm.lc1[te], c2 = dm.lc2[te];
    const T g0x = geo[te], g0y = geo[nte + te], g1x = geo[2 * nte + te], g1y = geo[3 * nte + te];
    const T g2x = geo[4 * nte + te], g2y = geo[5 * nte + te], A = geo[6 * nte + te];
    T exx, eyy, exy;
    elem_strain<T>(sux[c0], suy[c0], sux[c1], suy[c1], sux[c2], suy[c2], g0x, g0y, g1x, g1y, g2x, g2y, exx, eyy,
                   exy);
    T psi_p, sp[3], sm[3];
    split_eval<S, T>(exx, eyy, exy, P, psi_p, sp, sm);
    const double psi_m = 0.5 * (double(sm[0]) * exx + double(sm[1]) * eyy + 2.0 * double(sm[2]) * exy);
    const double d0 = sd[c0], d1 = sd[c1], d2 = sd[c2];
    const double ds = d0 + d1 + d2;
    const double om = 1.0 - ds / 3.0;
    const double gd = om * om + double(P.eta);
    ee += double(A) * (gd * double(psi_p) + psi_m);
    // d^e' K^e d^e = A |grad d|^2 and d^e' M^e d^e = A (sum d^2 + (sum d)^2) / 12
    const double gx = double(g0x) * d0 + double(g1x) * d1 + double(g2x) * d2;
    const double gy = double(g0y) * d0 + double(g1y) * d1 + double(g2y) * d2;
    const double dkd = double(A) * (gx * gx + gy * gy);
    const double first = at2 ? double(A) * (d0 * d0 + d1 * d1 + d2 * d2 + ds * ds) / 12.0 : double(A) * ds / 3.0;
    const double fe = double(P.efr) * (first + double(P.l0sq) * dkd);
    ef += gcs ? double(gcs[te]) * fe : fe;   // Gc_e = Gc phi_e
  }
  double v[3] = {ek, ee, ef};
  block_reduce_to0<3, 0u>(v, red);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) part[size_t(k) * dm.n_tiles + tile] = v[k];
  }
}

// One workgroup per instance: fixed-order sums of the tiles' partials.
__global__ __launch_bounds__(kBlock) void k_energy_reduce(const Ctl* ctl, const double* part, int n_tiles,
                                                          double* out) {
  __shared__ double red[3 * 4 * kWaves];
  const Ctl* c = ctl + blockIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = c->tile0 + threadIdx.x; k < c->tile0 + c->ntiles; k += kBlock) {
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] += part[size_t(j) * n_tiles + k];
  }
  block_reduce_to0<3, 0u>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) out[3 * blockIdx.x + j] = v[j];
  }
}

// Partials of pf_energies_static: a fixed array in device memory instead of
// the handle's workspace (one copy per device, alive until the process
// ends).  Host code never passes the array's name to a kernel: it uses the
// device address resolved by energy_scratch_setup.
static __device__ __align__(256) double scratch[3 * size_t(PF_ENERGY_STATIC_MAX_TILES)];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device; null until resolved
}  // namespace

pf_status_t energy_scratch_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return fail(PF_ERR_ARG, "invalid device");
  if (size_t(device) < g_scratch_ptr.size() && g_scratch_ptr[size_t(device)]) return PF_OK;
  double* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!ptr) return fail(PF_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
  if (g_scratch_ptr.size() <= size_t(device)) g_scratch_ptr.resize(size_t(device) + 1, nullptr);
  g_scratch_ptr[size_t(device)] = ptr;
  return PF_OK;
}

static double* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && size_t(device) < g_scratch_ptr.size()) ? g_scratch_ptr[size_t(device)] : nullptr;
}

template <typename T>
static pf_status_t energies_t(pf_mesh_s* m, int split, const pf_state_t* s, double* out, double* part,
                              hipStream_t st) {
  const dim3 grid(m->n_tiles), block(kBlock);
  const size_t lds = 3 * size_t(m->max_tile_nodes) * sizeof(T) + 64;
  const InstP<T>* ip = static_cast<const InstP<T>*>(m->dw.instp);
  const StateIn<T> si = state_in<T>(s);
  switch (split) {
    case SPLIT_NONE:
      hipLaunchKernelGGL((k_energy<T, SPLIT_NONE>), grid, block, lds, st, m->dm, ip, si, part);
      break;
    case SPLIT_SPECTRAL:
      hipLaunchKernelGGL((k_energy<T, SPLIT_SPECTRAL>), grid, block, lds, st, m->dm, ip, si, part);
      break;
    case SPLIT_VOLDEV:
      hipLaunchKernelGGL((k_energy<T, SPLIT_VOLDEV>), grid, block, lds, st, m->dm, ip, si, part);
      break;
    default:
      hipLaunchKernelGGL((k_energy<T, SPLIT_STAR>), grid, block, lds, st, m->dm, ip, si, part);
      break;
  }
  hipLaunchKernelGGL(k_energy_reduce, dim3(m->n_inst), block, 0, st, m->dw.ctl, part, m->n_tiles, out);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

}  // namespace pf

using namespace pf;

static pf_status_t energies_checked(pf_mesh_t m, const pf_params_t* p, const pf_state_t* s, double* out,
                                    pf_stream_t stream, bool fixed_scratch) {
  if (!m || !out) return fail(PF_ERR_ARG, "NULL argument");
  pf_status_t st;
  if ((st = check_params(m, p, nullptr, false)) != PF_OK) return st;
  if ((st = check_state(s, true, false, "state")) != PF_OK) return st;
  double* part = m->dw.part;
  if (fixed_scratch) {
    if (m->n_tiles > PF_ENERGY_STATIC_MAX_TILES)
      return fail(PF_ERR_ARG, "pf_energies_static: the handle has " + std::to_string(m->n_tiles) +
                                  " tiles, more than PF_ENERGY_STATIC_MAX_TILES = " +
                                  std::to_string(PF_ENERGY_STATIC_MAX_TILES) + "; use pf_energies");
    part = scratch_of(m->device);
    if (!part) return fail(PF_ERR_HIP, "pf_energies_static: no static partials resolved on this device");
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if ((st = upload_params(m, p, nullptr, hs)) != PF_OK) return st;
  return (m->dtype == PF_F64) ? energies_t<double>(m, p[0].split, s, out, part, hs)
                              : energies_t<float>(m, p[0].split, s, out, part, hs);
}

extern "C" pf_status_t pf_energies(pf_mesh_t m, const pf_params_t* p, const pf_state_t* s, double* out,
                                   pf_stream_t stream) {
  return energies_checked(m, p, s, out, stream, false);
}

extern "C" pf_status_t pf_energies_static(pf_mesh_t m, const pf_params_t* p, const pf_state_t* s, double* out,
                                          pf_stream_t stream) {
  return energies_checked(m, p, s, out, stream, true);
}
