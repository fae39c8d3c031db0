// Host-only dump of the pass descriptors that build_geometry produces, for
// the geometry tests (compiled with g++ by tests/test_plan_geometry.py).
// Usage: plan_dump n1 n2 n3 bc [p q r]
#include <cstdio>
#include <cstdlib>
#include <string>

#include "plan.h"

int main(int argc, char **argv) {
  if (argc != 5 && argc != 8) return 2;
  const int n1 = std::atoi(argv[1]), n2 = std::atoi(argv[2]), n3 = std::atoi(argv[3]);
  const unsigned bc = unsigned(std::atoi(argv[4]));
  int order[3];
  const int *force = nullptr;
  if (argc == 8) {
    for (int k = 0; k < 3; ++k) order[k] = std::atoi(argv[5 + k]);
    force = order;
  }
  psn::Geometry g;
  std::string err;
  const int rc = psn::build_geometry(n1, n2, n3, bc, g, err, force);
  if (rc) {
    std::printf("error %d %s\n", rc, err.c_str());
    return 0;
  }
  std::printf("geometry %d %d %d %d %d %d %lld %lld %d\n", g.order[0], g.order[1], g.order[2], g.S[0],
              g.S[1], g.S[2], g.a1_elems, g.a2_elems, int(psn::plane_geometry_ok(g)));
  for (int k = 0; k < 5; ++k) {
    const psn::Pass &P = g.pass[k];
    std::printf("pass %d %d %d %d %d %d %d %lld %lld %lld %lld %lld %lld %d %d %d %d\n", k, P.kind,
                P.L, P.n_in, P.n_out, P.ext_tile, P.ext_batch, P.in_s[0], P.in_s[1], P.in_s[2],
                P.out_s[0], P.out_s[1], P.out_s[2], int(P.in_tiled), int(P.out_tiled), int(P.pad),
                int(P.crop));
  }
  return 0;
}
