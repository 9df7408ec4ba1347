// Host-side paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (built by
// tests/test_sanitizers.py with g++, linked against the library's own objects): velocity
// sets of every order the library accepts (explicit and reduced), their node tables, state
// sizes, and the argument checks of init_state and step_noalloc, which all return before
// any device use.  Prints "ok" and exits 0 when every call returned what it should.
#include <cstdio>
#include <cstring>
#include <vector>

#include "hrlb.h"

static int failures = 0;
#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

int main() {
  for (int Qx = 1; Qx <= 128; Qx += (Qx < 16 ? 1 : 13)) {
    const int Nx = Qx - 1 < 6 ? Qx - 1 : 6;
    for (int Q = 1; Q <= 16; Q += 3) {
      hrlb_quad* q = nullptr;
      CHECK(hrlb_init_quadrature(Qx, Nx, Q, Q - 1, Q, Q - 1, &q) == HRLB_OK);
      int V = 0;
      CHECK(hrlb_quad_size(q, &V) == HRLB_OK && V == 2 * Qx * Q * Q);
      std::vector<double> p(2 * Qx), w(2 * Qx);
      CHECK(hrlb_quad_nodes(q, 0, p.data(), w.data()) == HRLB_OK);
      for (int i = 0; i < 2 * Qx; ++i) CHECK(p[i] == -p[2 * Qx - 1 - i]);
      std::vector<double> py(Q), wy(Q);
      CHECK(hrlb_quad_nodes(q, 1, py.data(), wy.data()) == HRLB_OK);
      CHECK(hrlb_quad_nodes(q, 3, py.data(), wy.data()) == HRLB_EINVAL);
      size_t sb = 0, wb = 0;
      CHECK(hrlb_state_bytes(q, 16, 3, &sb, &wb) == HRLB_OK && sb >= 3 * (size_t)3 * 16 * V * 8 && wb > 0);
      hrlb_quad_free(q);
      hrlb_quad* r = nullptr;
      CHECK(hrlb_init_quadrature_reduced(Qx, Nx, Q, Q - 1, &r) == HRLB_OK);
      CHECK(hrlb_quad_size(r, &V) == HRLB_OK && V == 4 * Qx * Q);
      CHECK(hrlb_quad_nodes(r, 2, py.data(), wy.data()) == HRLB_EINVAL);
      hrlb_quad_free(r);
    }
  }
  hrlb_quad* q = nullptr;
  CHECK(hrlb_init_quadrature(0, 0, 4, 3, 4, 3, &q) == HRLB_EINVAL && q == nullptr);
  CHECK(std::strlen(hrlb_last_error()) > 0);
  CHECK(hrlb_init_quadrature(8, 6, 4, 3, 4, 3, &q) == HRLB_OK);
  size_t sb = 0, wb = 0;
  CHECK(hrlb_state_bytes(q, 32, 2, &sb, &wb) == HRLB_OK);
  // fake device pointers: every call below fails its argument checks first
  void* fs = (void*)(uintptr_t)(1u << 20);
  void* fw = (void*)(uintptr_t)(1u << 30);
  hrlb_params par[2];
  std::memset(par, 0, sizeof(par));
  for (auto& x : par) {
    x.kn = 0.1;
    x.T_w = 1.0;
    x.n0 = 1.0;
    x.pr = 1.0;
    x.omega = 1.0;
    x.dt = 1e-3;
  }
  hrlb_sim* sim = nullptr;
  par[1].dt = 0.0;
  CHECK(hrlb_init_state(q, 32, HRLB_SCHEME_WENO5, par, 2, fs, sb, fw, wb, nullptr, nullptr, 0.0, &sim) == HRLB_EINVAL);
  par[1].dt = 1.0;  // beyond the RK3 stability limit of the advection
  CHECK(hrlb_init_state(q, 32, HRLB_SCHEME_WENO5, par, 2, fs, sb, fw, wb, nullptr, nullptr, 0.0, &sim) == HRLB_ENUMERIC);
  par[1].dt = 1e-3;
  CHECK(hrlb_init_state(q, 32, HRLB_SCHEME_WENO5, par, 2, fs, sb - 8, fw, wb, nullptr, nullptr, 0.0, &sim) == HRLB_ENOMEM);
  CHECK(hrlb_init_state(q, 2, HRLB_SCHEME_WENO5, par, 2, fs, sb, fw, wb, nullptr, nullptr, 0.0, &sim) == HRLB_EINVAL);
  CHECK(hrlb_init_state(q, 32, 9, par, 2, fs, sb, fw, wb, nullptr, nullptr, 0.0, &sim) == HRLB_EINVAL);
  CHECK(sim == nullptr);
  CHECK(hrlb_step_noalloc(q, 32, HRLB_SCHEME_WENO5, par, 2, fs, sb, -1, nullptr, nullptr) == HRLB_EINVAL);
  CHECK(hrlb_step_noalloc(q, 32, HRLB_SCHEME_WENO5, par, 2, fs, sb - 8, 1, nullptr, nullptr) == HRLB_ENOMEM);
  CHECK(hrlb_step(nullptr, 1) == HRLB_EINVAL);
  CHECK(hrlb_free_molecular_state(nullptr) == HRLB_EINVAL);
  hrlb_quad_free(q);
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
