// Spatially varying fracture toughness Gc_e = Gc phi_e (the per-element
// Gc(x) inverse problem named as the next step in Sec. 4).  The handle keeps
// phi in tile-element order next to the element geometry, so the damage,
// adjoint and energy kernels read it with the same coalesced index as the
// geometry; the adjoint can also accumulate dL/dGc_e per element.
#include <cmath>
#include <vector>

#include "device_common.hpp"

namespace pf {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gcs_gather(const int32_t* __restrict__ te_gid, const T* __restrict__ phi,
                                                       T* __restrict__ out, int n_te) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n_te) out[i] = phi[te_gid[i]];
}

template <typename T>
static pf_status_t check_field(const void* phi, int n, hipStream_t s) {
  std::vector<T> h(static_cast<size_t>(n));
  PF_HIP(hipMemcpyAsync(h.data(), phi, size_t(n) * sizeof(T), hipMemcpyDeviceToHost, s));
  PF_HIP(hipStreamSynchronize(s));
  for (int e = 0; e < n; ++e) {
    const double v = double(h[size_t(e)]);
    if (!std::isfinite(v) || !(v > 0.0))
      return fail(PF_ERR_ARG, "toughness factor of element " + std::to_string(e) + " is not finite and positive");
  }
  return PF_OK;
}

}  // namespace pf

using namespace pf;

extern "C" pf_status_t pf_set_gc_field(pf_mesh_t m, const void* phi, double* dgc_field, pf_stream_t stream) {
  if (!m) return fail(PF_ERR_ARG, "NULL mesh");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!phi) {
    m->dm.gcs = nullptr;
    m->dgc_field = dgc_field;
    return PF_OK;
  }
  const bool f64 = m->dtype == PF_F64;
  const size_t w = f64 ? sizeof(double) : sizeof(float);
  pf_status_t st = f64 ? check_field<double>(phi, m->n_elems, s) : check_field<float>(phi, m->n_elems, s);
  if (st != PF_OK) return st;
  if (!m->gcs_buf) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(size_t(m->n_te) * w, 16);
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(PF_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    m->allocs.push_back(p);   // freed with the handle
    m->device_bytes += bytes;
    m->gcs_buf = p;
  }
  const dim3 grid((m->n_te + kBlock - 1) / kBlock), block(kBlock);
  if (f64)
    hipLaunchKernelGGL(k_gcs_gather<double>, grid, block, 0, s, m->dm.te_gid, static_cast<const double*>(phi),
                       static_cast<double*>(m->gcs_buf), m->n_te);
  else
    hipLaunchKernelGGL(k_gcs_gather<float>, grid, block, 0, s, m->dm.te_gid, static_cast<const float*>(phi),
                       static_cast<float*>(m->gcs_buf), m->n_te);
  PF_HIP(hipGetLastError());
  // the caller may release phi on return
  PF_HIP(hipStreamSynchronize(s));
  m->dm.gcs = m->gcs_buf;
  m->dgc_field = dgc_field;
  return PF_OK;
}
