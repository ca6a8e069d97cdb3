// Host-side exercise of the hfmm C ABI for the sanitizer build: tree builds,
// the multi-threaded dual tree traversal and host plans (hfmm_tree_plan,
// hfmm_prepare_host) on several handles from several threads at once,
// structure exports, BIE and curved-element handles, the server's host
// half (create, submit, poll, free) and the argument checks.  Touches no
// device memory.  Usage: host_driver <points.f32> <ico.f64> <ico.i32>
// <curved.f64> <curved.i32> (flat binary arrays written by the test).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/hfmm.h"

template <class T>
static std::vector<T> load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", path);
    std::exit(2);
  }
  std::fseek(f, 0, SEEK_END);
  const long n = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<T> v(n / sizeof(T));
  if (std::fread(v.data(), sizeof(T), v.size(), f) != v.size()) std::exit(2);
  std::fclose(f);
  return v;
}

static int g_fail = 0;
#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__,   \
                   #cond, hfmm_last_error());                                \
      g_fail = 1;                                                            \
    }                                                                        \
  } while (0)

static void point_work(const std::vector<float>& xyz, int64_t n, double k, int P, int ncrit) {
  hfmm_opts o;
  hfmm_default_opts(&o);
  o.ncrit = ncrit;
  hfmm_tree* t = nullptr;
  CHECK(hfmm_build_tree(xyz.data(), n, &o, &t) == HFMM_OK);
  if (!t) return;
  hfmm_plan_info pi;
  CHECK(hfmm_tree_plan(t, k, P, 0, &pi) == HFMM_OK);
  int64_t fp = -1;
  CHECK(hfmm_prepare_host(t, k, P, &fp) == HFMM_OK && fp == pi.bytes_total);
  hfmm_stats st;
  CHECK(hfmm_tree_stats(t, k, P, &st) == HFMM_OK && st.n_m2l == pi.n_m2l);
  std::vector<int32_t> m2l(2 * st.n_m2l + 2), p2p(2 * st.n_p2p + 2);
  CHECK(hfmm_lists_export(t, k, P, m2l.data(), p2p.data()) == HFMM_OK);
  std::vector<int32_t> sp(st.n_src), tp(st.n_tgt), cells(10 * (size_t)st.n_cell);
  CHECK(hfmm_tree_export(t, k, P, sp.data(), tp.data(), cells.data()) == HFMM_OK);
  // a second (k, P) on the same handle, and the base tree
  CHECK(hfmm_tree_plan(t, 0.5 * k, P > 2 ? P - 2 : P, 0, &pi) == HFMM_OK);
  CHECK(hfmm_tree_export(t, 1.0, 0, sp.data(), nullptr, nullptr) == HFMM_OK);
  hfmm_tree_free(t);
}

// The matrix-core M2L's code tables (library internals, host side): for every
// order, each reflection maps the P^2 target coefficients to distinct
// staging positions inside a slot, and every input code addresses an
// aligned pair inside a multipole (the builder checks that x and y are one
// pair and throws otherwise).
namespace hfmm {
void m2l_xz_codes(int P, std::vector<int32_t>& in, std::vector<int32_t>& out);
void stage_dims(int P, int* Sm, int* St);
}  // namespace hfmm

static void code_tables() {
  for (int P = 1; P <= 16; ++P) {
    std::vector<int32_t> in, out;
    hfmm::m2l_xz_codes(P, in, out);
    int Sm = 0, St = 0;
    hfmm::stage_dims(P, &Sm, &St);
    const int P2 = P * P;
    CHECK((int)out.size() == 16 * P2);
    CHECK(Sm + St >= P2 && Sm % 16 == 0 && St % 2 == 0);
    for (int g = 0; g < 16; ++g) {
      std::vector<char> seen(Sm + St, 0);
      for (int c = 0; c < P2; ++c) {
        const int pos = out[(size_t)g * P2 + c] & 0xffff;
        CHECK(pos >= 0 && pos < Sm + St && !seen[pos]);
        if (pos >= 0 && pos < Sm + St) seen[pos] = 1;
      }
    }
    // the input codes ([17][stride], then 16 ceil(S/16) m' entries): an even
    // base inside the multipole, and for even P^2 the whole pair inside it
    const int S = P * (P - 1) / 2, mrows = 16 * ((S + 15) / 16);
    CHECK((in.size() - mrows) % 17 == 0);
    for (size_t i = 0; i + mrows < in.size(); ++i) {
      const int base = in[i] & 0xff;
      CHECK(base % 2 == 0 && base < P2 && (P2 % 2 == 1 || base + 1 < P2));
    }
  }
}

int main(int argc, char** argv) {
  code_tables();
  if (argc != 6) {
    std::fprintf(stderr, "usage: host_driver points.f32 ico.f64 ico.i32 curved.f64 curved.i32\n");
    return 2;
  }
  const std::vector<float> pts = load<float>(argv[1]);
  const int64_t n = (int64_t)pts.size() / 3;
  // point handles from several threads at once, each plan itself threaded
  {
    std::vector<std::thread> th;
    const double ks[4] = {1.0, 30.0, 50.265482457, 8.0};
    const int Ps[4] = {8, 10, 10, 6};
    const int64_t ns[4] = {n, n / 2, n, 3001};
    for (int i = 0; i < 4; ++i)
      th.emplace_back(point_work, std::cref(pts), ns[i], ks[i], Ps[i], i == 3 ? 17 : 64);
    for (auto& x : th) x.join();
  }
  // flat BIE handle: host plan and the server's host half
  const std::vector<double> V = load<double>(argv[2]);
  const std::vector<int32_t> T = load<int32_t>(argv[3]);
  hfmm_tree* b = nullptr;
  CHECK(hfmm_build_bie(V.data(), (int64_t)V.size() / 3, T.data(), (int64_t)T.size() / 3, nullptr, &b) == HFMM_OK);
  if (b) {
    hfmm_plan_info pi;
    CHECK(hfmm_tree_plan(b, 6.0, 10, 30, &pi) == HFMM_OK && pi.bytes_gmres > 0 && pi.n_near > 0);
    hfmm_server* sv = nullptr;
    CHECK(hfmm_server_create(0, 4, &sv) == HFMM_OK);
    CHECK(hfmm_server_set_limits(sv, 3, 0.5, 10.0) == HFMM_OK);
    CHECK(hfmm_server_set_limits(sv, -1, 0.5, 0.0) == HFMM_EINVAL);
    int64_t ticket = 0, foot = 0;
    // dummy device pointers are never dereferenced: the solve stays queued
    void* fake = reinterpret_cast<void*>(0x1000);
    CHECK(hfmm_server_submit(sv, b, 6.0, 10, fake, fake, 1e-4, 30, 100, &ticket, &foot) == HFMM_OK);
    CHECK(foot >= pi.bytes_gmres);
    int64_t t2;
    CHECK(hfmm_server_submit(sv, b, 6.0, 10, fake, fake, 1e-4, 30, 100, &t2, nullptr) == HFMM_EINVAL);
    int32_t state = -9;
    hfmm_gmres_info info;
    double times[3];
    CHECK(hfmm_server_poll(sv, ticket, &state, &info, times) == HFMM_OK && state == 0);
    CHECK(hfmm_server_release(sv, ticket) == HFMM_EINVAL);
    CHECK(hfmm_server_poll(sv, ticket + 99, &state, nullptr, nullptr) == HFMM_EINVAL);
    hfmm_server_free(sv);
    hfmm_tree_free(b);
  }
  // curved-element handle
  const std::vector<double> N6 = load<double>(argv[4]);
  const std::vector<int32_t> T6 = load<int32_t>(argv[5]);
  hfmm_tree* c = nullptr;
  CHECK(hfmm_build_nystrom(N6.data(), (int64_t)N6.size() / 3, T6.data(), (int64_t)T6.size() / 6, nullptr, &c) ==
        HFMM_OK);
  if (c) {
    const int64_t np = 6 * ((int64_t)T6.size() / 6);
    std::vector<double> xyz(3 * np), w(np), jac(np);
    CHECK(hfmm_nystrom_points(c, xyz.data(), w.data(), jac.data()) == HFMM_OK);
    hfmm_plan_info pi;
    CHECK(hfmm_tree_plan(c, 2 * M_PI, 10, 30, &pi) == HFMM_OK && pi.n_src == np);
    hfmm_tree_free(c);
  }
  // argument checks
  hfmm_tree* t = nullptr;
  CHECK(hfmm_build_tree(pts.data(), 0, nullptr, &t) == HFMM_EINVAL && t == nullptr);
  std::vector<int32_t> bad(T.begin(), T.end());
  bad[4] = 1 << 29;
  CHECK(hfmm_build_bie(V.data(), (int64_t)V.size() / 3, bad.data(), (int64_t)bad.size() / 3, nullptr, &t) ==
        HFMM_EINVAL);
  CHECK(hfmm_tree_plan(nullptr, 1.0, 8, 0, nullptr) == HFMM_EINVAL);
  CHECK(hfmm_debug_fail_alloc(-2) == HFMM_EINVAL);
  std::printf("host driver: %s\n", g_fail ? "FAILED" : "ok");
  return g_fail;
}
