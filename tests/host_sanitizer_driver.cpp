// Host-side driver for the sanitizer build of the library (see
// test_host_sanitizers.py): mesh creation on valid and invalid inputs, so
// that the host code (validation, geometry, recursive bisection, tile plan,
// error paths) runs under AddressSanitizer and UndefinedBehaviorSanitizer.
// Without a GPU a valid mesh stops at the first device allocation, after the
// whole tile plan has been built on the host.
#include <cstdio>
#include <vector>

#include "pf.h"

namespace {

struct Grid {
  std::vector<double> xy;
  std::vector<int32_t> tri;
  std::vector<uint8_t> fixed;
};

Grid grid(int nx, int ny, unsigned seed) {
  Grid g;
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i <= nx; ++i) {
      seed = seed * 1103515245u + 12345u;
      const double jx = double((seed >> 16) % 1000) / 1000.0 - 0.5;
      seed = seed * 1103515245u + 12345u;
      const double jy = double((seed >> 16) % 1000) / 1000.0 - 0.5;
      const bool edge = i == 0 || j == 0 || i == nx || j == ny;
      g.xy.push_back(i + (edge ? 0.0 : 0.2 * jx));
      g.xy.push_back(j + (edge ? 0.0 : 0.2 * jy));
      g.fixed.push_back(j == 0 || j == ny ? 2 : 0);
      g.fixed.push_back(0);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int a = j * (nx + 1) + i, b = a + 1, c = a + nx + 1, d = c + 1;
      if ((i + j) % 3 == 0)
        g.tri.insert(g.tri.end(), {a, b, c, b, d, c});
      else
        g.tri.insert(g.tri.end(), {a, d, b, a, c, d});   // clockwise: the library reorients
    }
  return g;
}

pf_mesh_desc_t desc(const Grid& g) {
  return pf_mesh_desc_t{int32_t(g.xy.size() / 2), int32_t(g.tri.size() / 3), g.xy.data(), g.tri.data(),
                        g.fixed.data()};
}

void create(const char* name, const pf_mesh_desc_t* d, int n, pf_dtype_t dt, int tile) {
  pf_tile_opts_t o{tile, 0, 0, 0};
  pf_mesh_t m = nullptr;
  const pf_status_t st = pf_mesh_create(d, n, dt, &o, nullptr, &m);
  std::printf("%s %d\n", name, int(st));
  if (m) pf_mesh_destroy(m);
}

}  // namespace

int main() {
  const Grid a = grid(48, 24, 1), b = grid(33, 17, 2);
  const pf_mesh_desc_t da = desc(a), db = desc(b);
  create("valid_f64_t64", &da, 1, PF_F64, 64);
  create("valid_f32_t256", &da, 1, PF_F32, 256);
  create("valid_f64_t2048", &da, 1, PF_F64, 2048);
  const pf_mesh_desc_t two[2] = {da, db};
  create("valid_batched", two, 2, PF_F32, 128);
  // invalid inputs, each refused on the host
  Grid z = a;
  z.xy[2 * z.tri[4]] = z.xy[2 * z.tri[3]];          // second triangle: two corners at one point
  z.xy[2 * z.tri[4] + 1] = z.xy[2 * z.tri[3] + 1];
  const pf_mesh_desc_t dz = desc(z);
  create("zero_area", &dz, 1, PF_F64, 64);
  Grid r = a;
  r.tri[7] = int32_t(r.xy.size() / 2);               // node id out of range
  const pf_mesh_desc_t dr = desc(r);
  create("index_range", &dr, 1, PF_F64, 64);
  Grid u = a;
  u.xy.push_back(100.0);                             // a node in no element
  u.xy.push_back(100.0);
  u.fixed.push_back(0);
  u.fixed.push_back(0);
  const pf_mesh_desc_t du = desc(u);
  create("unused_node", &du, 1, PF_F64, 64);
  create("no_instances", &da, 0, PF_F64, 64);
  create("tile_too_large", &da, 1, PF_F64, 5000);
  return 0;
}
