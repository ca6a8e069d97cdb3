// Host-side octree, Morton keys and dual tree traversal (Sec. 2.3, 3.1, 3.2).
//
// The tree is built once per geometry in deterministic FP64 from the FP32
// coordinates; every decision uses exact dyadic or integer arithmetic, so the
// lists are reproducible bit for bit.  Readings of the unspecified details:
//  - root cube: he = max half-extent of all points (1 if 0); q = largest power
//    of two <= he/64; centre = nearest multiple of q to the bbox midpoint
//    (floor(mid/q + 0.5) q); half-width H = smallest power of two >= q with
//    |x - c| < H on every axis;
//  - keys: floor(((x - c) + H) / (2H) * 2^21) per axis, clamped, interleaved
//    with x in the lowest bit; stable sort (ties keep input order);
//  - a cell splits into its non-empty octants when it holds more than ncrit
//    sources, or (per wavenumber) when it is non-empty and wider than kappa/k,
//    since such a cell can never take part in M2L; cells are stored level by
//    level in Morton order;
//  - acceptance for M2L: 3 (sA + sB)^2 < theta^2 D2 (half-sides and squared
//    centre distance in units of the finer half-side) and k * side <= kappa
//    for the larger cell; traversal from (root, root) splits the cell with
//    the larger radius (ties: the target), or the other one if it is a leaf.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <atomic>
#include <map>
#include <mutex>
#include <numeric>
#include <stdexcept>

#include "hfmm_internal.h"

namespace hfmm {

static void root_cube(const float* a, int64_t na, const float* b, int64_t nb, double c[3],
                      double& H) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  auto scan = [&](const float* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) {
        double v = (double)p[3 * i + d];
        lo[d] = std::min(lo[d], v);
        hi[d] = std::max(hi[d], v);
      }
  };
  scan(a, na);
  if (b) scan(b, nb);
  double he = 0.0;
  for (int d = 0; d < 3; ++d) he = std::max(he, (hi[d] - lo[d]) / 2.0);
  if (he == 0.0) he = 1.0;
  double q = std::ldexp(1.0, (int)std::floor(std::log2(he / 64.0)));
  while (q * 2.0 <= he / 64.0) q *= 2.0;
  while (q > he / 64.0) q /= 2.0;
  for (int d = 0; d < 3; ++d) c[d] = std::floor(((lo[d] + hi[d]) / 2.0) / q + 0.5) * q;
  H = q;
  auto inside = [&](const float* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d)
        if (!(std::fabs((double)p[3 * i + d] - c[d]) < H)) return false;
    return true;
  };
  while (!(inside(a, na) && (!b || inside(b, nb)))) H *= 2.0;
}

static uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
  uint64_t r = 0;
  for (int b = 0; b < kKeyBits; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

static void keys_of(const float* p, int64_t n, const double c[3], double H,
                    std::vector<uint64_t>& key) {
  key.resize(n);
  const double scale = double(1u << kKeyBits);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = 0;
    for (int d = 0; d < 3; ++d) {
      double f = std::floor((((double)p[3 * i + d] - c[d]) + H) / (2.0 * H) * scale);
      int64_t kd = (int64_t)f;
      kd = std::min<int64_t>(std::max<int64_t>(kd, 0), (1 << kKeyBits) - 1);
      k |= spread3((uint64_t)kd) << d;
    }
    key[i] = k;
  }
}

static void sort_by_key(const std::vector<uint64_t>& key, std::vector<int32_t>& perm) {
  perm.resize(key.size());
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int32_t x, int32_t y) { return key[x] < key[y]; });
}

void build_tree(const float* src, int64_t nsrc, const float* tgt, int64_t ntgt, int ncrit,
                int max_level, HostTree& t) {
  t = HostTree();
  t.point_mode = (tgt == nullptr);
  t.nsrc = nsrc;
  t.ntgt = t.point_mode ? nsrc : ntgt;
  t.ncrit = ncrit;
  root_cube(src, nsrc, tgt, t.point_mode ? 0 : ntgt, t.c, t.H);
  std::vector<uint64_t> skey, tkey;
  keys_of(src, nsrc, t.c, t.H, skey);
  sort_by_key(skey, t.src_perm);
  t.skey.resize(nsrc);
  for (int64_t i = 0; i < nsrc; ++i) t.skey[i] = skey[t.src_perm[i]];
  if (t.point_mode) {
    t.tgt_perm = t.src_perm;
  } else {
    keys_of(tgt, ntgt, t.c, t.H, tkey);
    sort_by_key(tkey, t.tgt_perm);
    t.tkey.resize(ntgt);
    for (int64_t i = 0; i < ntgt; ++i) t.tkey[i] = tkey[t.tgt_perm[i]];
  }
  t.src_xyz.resize(3 * nsrc);
  for (int64_t i = 0; i < nsrc; ++i)
    for (int d = 0; d < 3; ++d) t.src_xyz[3 * i + d] = src[3 * (int64_t)t.src_perm[i] + d];
  if (t.point_mode) {
    t.tgt_xyz = t.src_xyz;
  } else {
    t.tgt_xyz.resize(3 * ntgt);
    for (int64_t i = 0; i < ntgt; ++i)
      for (int d = 0; d < 3; ++d) t.tgt_xyz[3 * i + d] = tgt[3 * (int64_t)t.tgt_perm[i] + d];
  }
  build_cells(t, ncrit, max_level, INFINITY, t);
}

void build_cells(const HostTree& b, int ncrit, int max_level, double split_side, HostTree& t) {
  const std::vector<uint64_t>& sk = b.skey;
  const std::vector<uint64_t>& tk = b.point_mode ? b.skey : b.tkey;
  if (&t != &b) {
    t.point_mode = b.point_mode;
    t.nsrc = b.nsrc;
    t.ntgt = b.ntgt;
    for (int d = 0; d < 3; ++d) t.c[d] = b.c[d];
    t.H = b.H;
  }
  t.ncrit = ncrit;
  t.level.clear(); t.ijk.clear(); t.sb.clear(); t.se.clear(); t.tb.clear(); t.te.clear();
  t.cb.clear(); t.ce.clear(); t.parent.clear(); t.level_off.clear();
  auto push = [&](int lev, int i, int j, int k, int32_t a, int32_t bb, int32_t c0, int32_t d,
                  int32_t par) {
    t.level.push_back(lev);
    t.ijk.push_back(i);
    t.ijk.push_back(j);
    t.ijk.push_back(k);
    t.sb.push_back(a);
    t.se.push_back(bb);
    t.tb.push_back(c0);
    t.te.push_back(d);
    t.cb.push_back(0);
    t.ce.push_back(0);
    t.parent.push_back(par);
  };
  push(0, 0, 0, 0, 0, (int32_t)t.nsrc, 0, (int32_t)t.ntgt, -1);
  std::vector<int32_t> cur = {0}, nxt;
  int lev = 0;
  while (!cur.empty()) {
    nxt.clear();
    const double side = 2.0 * t.H / double(1 << lev);
    for (int32_t ci : cur) {
      int32_t ns = t.se[ci] - t.sb[ci];
      int32_t nb = t.point_mode ? ns : ns + (t.te[ci] - t.tb[ci]);
      bool force = side > split_side && nb >= 1;
      if ((ns <= ncrit && !force) || lev >= max_level) {
        t.cb[ci] = t.ce[ci] = (int32_t)t.level.size();
        continue;
      }
      int shift = 3 * (kKeyBits - lev - 1);
      int32_t first = (int32_t)t.level.size();
      int32_t s0 = t.sb[ci], t0 = t.tb[ci];
      for (int o = 0; o < 8; ++o) {
        auto oct = [&](uint64_t key) { return (int)((key >> shift) & 7ull); };
        int32_t s1 = s0, t1 = t0;
        while (s1 < t.se[ci] && oct(sk[s1]) == o) ++s1;
        while (t1 < t.te[ci] && oct(tk[t1]) == o) ++t1;
        if (s1 > s0 || t1 > t0) {
          int i = t.ijk[3 * ci], j = t.ijk[3 * ci + 1], k = t.ijk[3 * ci + 2];
          push(lev + 1, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + ((o >> 2) & 1), s0, s1,
               t0, t1, ci);
          nxt.push_back((int32_t)t.level.size() - 1);
        }
        s0 = s1;
        t0 = t1;
      }
      t.cb[ci] = first;
      t.ce[ci] = (int32_t)t.level.size();
    }
    cur.swap(nxt);
    ++lev;
  }
  t.level_off.push_back(0);
  for (int i = 1; i < t.ncell(); ++i)
    if (t.level[i] != t.level[i - 1]) t.level_off.push_back(i);
  t.level_off.push_back(t.ncell());
}

static inline bool mac(const HostTree& t, int a, int b, double k, double theta,
                       double kappa) {
  int la = t.level[a], lb = t.level[b];
  int L = std::max(la, lb);
  int64_t D2 = 0;
  for (int d = 0; d < 3; ++d) {
    int64_t ca = -(int64_t(1) << L) + (2 * (int64_t)t.ijk[3 * a + d] + 1) * (int64_t(1) << (L - la));
    int64_t cb = -(int64_t(1) << L) + (2 * (int64_t)t.ijk[3 * b + d] + 1) * (int64_t(1) << (L - lb));
    D2 += (ca - cb) * (ca - cb);
  }
  int64_t sA = int64_t(1) << (L - la), sB = int64_t(1) << (L - lb);
  bool geo = 3.0 * double((sA + sB) * (sA + sB)) < (theta * theta) * double(D2);
  double hmax = t.H / double(1 << std::min(la, lb));
  return geo && (k * (2.0 * hmax) <= kappa);
}

// Serial depth-first traversal of the pair (a0, b0), appending to out: the
// stack pops children in the order they are stored.
static void dtt_from(const HostTree& t, int32_t a0, int32_t b0, double k, double theta, double kappa,
                     Lists& out) {
  std::vector<std::pair<int32_t, int32_t>> stack;
  stack.reserve(4096);
  stack.push_back({a0, b0});
  while (!stack.empty()) {
    auto [a, b] = stack.back();
    stack.pop_back();
    if (t.te[a] == t.tb[a] || t.se[b] == t.sb[b]) continue;
    if (mac(t, a, b, k, theta, kappa)) {
      out.m2l_a.push_back(a);
      out.m2l_b.push_back(b);
      continue;
    }
    bool la = t.leaf(a), lb = t.leaf(b);
    if (la && lb) {
      out.p2p_a.push_back(a);
      out.p2p_b.push_back(b);
      continue;
    }
    bool split_a = !la && (t.level[a] <= t.level[b] || lb);
    if (split_a) {
      for (int ch = t.ce[a] - 1; ch >= t.cb[a]; --ch) stack.push_back({ch, b});
    } else {
      for (int ch = t.ce[b] - 1; ch >= t.cb[b]; --ch) stack.push_back({a, ch});
    }
  }
}

// The traversal from (root, root).  The first levels are expanded into a
// frontier in depth-first order (finished pairs stay in place); the frontier's
// subtrees are then traversed on several threads and their lists appended in
// frontier order, which is exactly the serial depth-first order.
void dual_tree_traversal(const HostTree& t, double k, double theta, double kappa, Lists& out) {
  out = Lists();
  const int T = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  struct Item {
    int32_t a, b;
    int8_t kind;  // 0 open, 1 M2L, 2 P2P, 3 empty
  };
  std::vector<Item> front{{0, 0, 0}};
  for (int round = 0; round < 12; ++round) {
    size_t open = 0;
    for (const Item& it : front) open += it.kind == 0;
    if (open == 0 || open >= (size_t)64 * T) break;
    std::vector<Item> next;
    next.reserve(front.size() * 8);
    for (const Item& it : front) {
      if (it.kind != 0) {
        next.push_back(it);
        continue;
      }
      const int32_t a = it.a, b = it.b;
      if (t.te[a] == t.tb[a] || t.se[b] == t.sb[b]) continue;
      if (mac(t, a, b, k, theta, kappa)) {
        next.push_back({a, b, 1});
        continue;
      }
      bool la = t.leaf(a), lb = t.leaf(b);
      if (la && lb) {
        next.push_back({a, b, 2});
        continue;
      }
      bool split_a = !la && (t.level[a] <= t.level[b] || lb);
      if (split_a) {
        for (int ch = t.cb[a]; ch < t.ce[a]; ++ch) next.push_back({ch, b, 0});
      } else {
        for (int ch = t.cb[b]; ch < t.ce[b]; ++ch) next.push_back({a, ch, 0});
      }
    }
    front.swap(next);
  }
  std::vector<Lists> part(front.size());
  std::atomic<size_t> cursor{0};
  auto work = [&]() {
    for (size_t i; (i = cursor.fetch_add(1)) < front.size();) {
      const Item& it = front[i];
      if (it.kind == 0) dtt_from(t, it.a, it.b, k, theta, kappa, part[i]);
    }
  };
  std::vector<std::thread> th;
  for (int i = 1; i < T; ++i) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
  for (size_t i = 0; i < front.size(); ++i) {
    const Item& it = front[i];
    if (it.kind == 1) {
      out.m2l_a.push_back(it.a);
      out.m2l_b.push_back(it.b);
    } else if (it.kind == 2) {
      out.p2p_a.push_back(it.a);
      out.p2p_b.push_back(it.b);
    } else if (it.kind == 0) {
      const Lists& L = part[i];
      out.m2l_a.insert(out.m2l_a.end(), L.m2l_a.begin(), L.m2l_a.end());
      out.m2l_b.insert(out.m2l_b.end(), L.m2l_b.begin(), L.m2l_b.end());
      out.p2p_a.insert(out.p2p_a.end(), L.p2p_a.begin(), L.p2p_a.end());
      out.p2p_b.insert(out.p2p_b.end(), L.p2p_b.begin(), L.p2p_b.end());
    }
  }
}

// ---------------------------------------------------------------------------
// Gaunt coupling: integral of Y_n^m conj(Y_n'^m') conj(Y_l^{m-m'}) over the
// sphere, with the phi integral done exactly (2 pi) and the cos(theta)
// integral by Gauss-Legendre quadrature, exact for the polynomial integrand of
// degree n + n' + l <= 4P - 4.
// ---------------------------------------------------------------------------
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Normalised associated Legendre values pbar_n^m(x) (no Condon-Shortley
// phase, orthonormal with the 1/(4 pi) of Y) for n < L, m <= n.
static void legendre_norm(int L, double x, std::vector<double>& p) {
  p.assign(L * L, 0.0);
  double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  auto at = [&](int n, int m) -> double& { return p[n * n + n + m]; };
  at(0, 0) = 1.0 / std::sqrt(4.0 * M_PI);
  for (int m = 1; m < L; ++m) at(m, m) = std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * at(m - 1, m - 1);
  for (int m = 0; m + 1 < L; ++m) at(m + 1, m) = std::sqrt(2.0 * m + 3.0) * x * at(m, m);
  for (int m = 0; m < L; ++m)
    for (int n = m + 2; n < L; ++n) {
      double a = std::sqrt((4.0 * n * n - 1.0) / (double(n) * n - double(m) * m));
      double b = std::sqrt((double(n - 1) * (n - 1) - double(m) * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
      at(n, m) = a * (x * at(n - 1, m) - b * at(n - 2, m));
    }
}

const Coupling& coupling(int P) {
  // shared by every handle: handles may be prepared from several threads at
  // once (entries are never removed, so references stay valid)
  static std::mutex mu;
  static std::map<int, Coupling> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(P);
  if (it != cache.end()) return it->second;
  Coupling cp;
  cp.P = P;
  int L = 2 * P - 1;  // harmonic degrees 0..2P-2
  int ng = 2 * P + 2;
  std::vector<double> gx, gw;
  gauss_legendre(ng, gx, gw);
  std::vector<std::vector<double>> pl(ng);
  for (int i = 0; i < ng; ++i) legendre_norm(L, gx[i], pl[i]);
  auto pbar = [&](int g, int n, int m) { return pl[g][n * n + n + std::abs(m)]; };
  int P2 = P * P;
  cp.off.assign(P2 * P2 + 1, 0);
  for (int n2 = 0; n2 < P; ++n2)
    for (int m2 = -n2; m2 <= n2; ++m2) {
      int row = n2 * n2 + n2 + m2;
      for (int n = 0; n < P; ++n)
        for (int m = -n; m <= n; ++m) {
          int col = n * n + n + m;
          int mu = m - m2;
          for (int l = std::abs(n - n2); l <= n + n2; ++l) {
            if (std::abs(mu) > l || ((n + n2 + l) & 1)) continue;
            double g = 0.0;
            for (int q = 0; q < ng; ++q) g += gw[q] * pbar(q, n, m) * pbar(q, n2, m2) * pbar(q, l, mu);
            g *= 2.0 * M_PI;
            if (std::fabs(g) < 1e-15) continue;
            int e = ((n2 + l - n) % 4 + 4) % 4;  // i^e
            double re = (e == 0 ? 1.0 : e == 2 ? -1.0 : 0.0) * 4.0 * M_PI * g;
            double im = (e == 1 ? 1.0 : e == 3 ? -1.0 : 0.0) * 4.0 * M_PI * g;
            cp.lm.push_back(l * l + l + mu);
            cp.re.push_back(re);
            cp.im.push_back(im);
          }
          cp.off[row * P2 + col + 1] = (int32_t)cp.lm.size();
        }
    }
  auto res = cache.emplace(P, std::move(cp));
  return res.first->second;
}

// Reflection g = bits (fx, fy, fz, swap x<->y) of the cube acts on the
// harmonics as Y_n^m(sigma r) = i^ph Y_n^{m'}(r): x -> -x gives m' = -m and
// ph = 2m; y -> -y gives m' = -m; z -> -z gives ph = 2(n + m); the x<->y
// swap gives m' = -m and ph = m; g applies them in that order.  For a pair
// translated through the canonical operator, the input row k = (n, m') takes
// B[k] = i^ph M[c] with c = (n, m), and the output row k goes back to c as
// L[c] += i^-ph C[k].
static int32_t phase_code(int idx, int ph) {
  // i^ph (x + iy): 0 -> (x, y), 1 -> (-y, x), 2 -> (-x, -y), 3 -> (y, -x)
  const uint32_t swap = ph & 1, neg_re = (ph == 1 || ph == 2), neg_im = ph >= 2;
  return (int32_t)((uint32_t)idx | swap << 16 | neg_im << 30 | neg_re << 31);
}

void m2l_reflection_codes(int P, int Kp, std::vector<int32_t>& in, std::vector<int32_t>& out) {
  const int P2 = P * P;
  in.assign(17 * (size_t)Kp, 1 << 17);
  out.assign(16 * (size_t)P2, 0);
  for (int g = 0; g < 16; ++g)
    for (int n = 0; n < P; ++n)
      for (int m = -n; m <= n; ++m) {
        int cm = m, ph = 0;
        if (g & 1) { ph += 2 * std::abs(cm % 2); cm = -cm; }
        if (g & 2) { cm = -cm; }
        if (g & 4) { ph += 2 * std::abs((n + cm) % 2); }
        if (g & 8) { ph += ((cm % 4) + 4) % 4; cm = -cm; }
        ph &= 3;
        const int k = n * n + n + cm;   // row in the canonical frame
        const int c = n * n + n + m;
        in[(size_t)g * Kp + k] = phase_code(c, ph);
        out[(size_t)g * P2 + c] = phase_code(k, (4 - ph) & 3);
      }
}


// Codes of the xz-plane M2L (XzDims).  in: [17][xz_code_stride(P)], for
// reflection g and C-list input k = (n, m), one word telling where the two
// reflected multipoles B[(n, m)] = i^a M[(n, s m)] (x) and B[(n, -m)] =
// i^b M[(n, -s m)] (y) are found and how to turn them.  The source's
// multipole is stored in mpos order, so one aligned pair of float2 at
// `base` holds lo = M[(n, |m|)] and hi = M[(n, -|m|)]; s = -1 when g flips
// the sign of m, and then x is hi:
//   bits 0..7 base (even), 8 conj (s = -1, m > 0), 9..12 m,
//   lo's phase: 16 swap, 17 zero, 30 neg_im, 31 neg_re,
//   hi's phase: 13 swap, 14 zero, 27 neg_im, 28 neg_re
// (the word shifted left by 3 carries hi's flags where lo's are).  With
// p = e^{i m phi} and q = conj(p) if conj else p, the kernel forms
//   u = q lo' + conj(q) hi',  v = q lo' - conj(q) hi'
// from the turned lo', hi', which equals p x + conj(p) y and, up to the
// sign s of the whole column, p x - conj(p) y.  For m = 0, x is lo or hi of
// the pair holding (n, 0) and the other is marked zero; for k >= C both.
// Row 16 (columns past a chunk's end) has both marked zero.  Then 16 RTS
// entries: m' of S-list output row r (0 past the list).  out: [16][P^2],
// for target coefficient c = (n, m) under reflection g: the staging position
// of the canonical (n, m') it comes from (xz_stage_pos) and the phase i^-ph
// (swap bit 16, signs in bits 30, 31).
void m2l_xz_codes(int P, std::vector<int32_t>& in, std::vector<int32_t>& out) {
  const XzDims d = xz_dims(P);
  const int P2 = P * P, Kp = 4 * ((P2 + 3) / 4);
  const uint32_t zlo = 1u << 17, zhi = 1u << 14;
  const uint32_t lo_ph = (1u << 16) | (3u << 30);  // a dense code's phase bits, in lo's place
  std::vector<int32_t> dense_in, dense_out;
  m2l_reflection_codes(P, Kp, dense_in, dense_out);
  // storage position of standard index c = n^2 + n + m
  std::vector<int> pos(P2);
  for (int n = 0; n < P; ++n)
    for (int m = -n; m <= n; ++m) pos[n * n + n + m] = mpos(P, n, m);
  const int ks = xz_code_stride(P);
  in.assign(17 * (size_t)ks + 16 * (size_t)d.RTS, (int32_t)(zlo | zhi));
  for (int g = 0; g < 17; ++g)
    for (int e = 0; e < d.C; ++e) {
      int n, m;
      xz_entry(P, e, &n, &m);
      uint32_t w = (uint32_t)m << 9;
      if (g == 16) {
        w |= zlo | zhi;
      } else {
        const uint32_t dx = (uint32_t)dense_in[(size_t)g * Kp + n * n + n + m];
        const int px = pos[dx & 0xffff];
        const bool xhi = px & 1;
        w |= (uint32_t)(px & ~1);
        if (m > 0) {
          const uint32_t dy = (uint32_t)dense_in[(size_t)g * Kp + n * n + n - m];
          if ((pos[dy & 0xffff] ^ px) != 1) throw std::logic_error("M2L code table: x and y not one pair");
          const uint32_t clo = xhi ? dy : dx, chi = xhi ? dx : dy;
          w |= (clo & lo_ph) | ((chi & lo_ph) >> 3) | (xhi ? 1u << 8 : 0u);
        } else {
          // x alone, in lo's or hi's place
          w |= xhi ? (((dx & lo_ph) >> 3) | zlo) : ((dx & lo_ph) | zhi);
        }
      }
      in[(size_t)g * ks + e] = (int32_t)w;
    }
  int32_t* mrow = in.data() + 17 * (size_t)ks;
  for (int r = 0; r < 16 * d.RTS; ++r) {
    int n = 0, m = 0;
    if (r < d.S) xz_entry(P, r, &n, &m);
    mrow[r] = m;
  }
  // staging position of each canonical coefficient (n, m')
  std::vector<int32_t> srow(P2, -1);
  for (int e = 0; e < d.C; ++e) {
    int n, m;
    xz_entry(P, e, &n, &m);
    srow[n * n + n + m] = xz_stage_pos(P, e, 1);
    if (m > 0) srow[n * n + n - m] = xz_stage_pos(P, e, -1);
  }
  out.assign(16 * (size_t)P2, 0);
  for (int g = 0; g < 16; ++g)
    for (int c = 0; c < P2; ++c) {
      const int32_t code = dense_out[(size_t)g * P2 + c];  // canonical row in bits 0..15, phase above
      out[(size_t)g * P2 + c] = (code & ~0xffff) | srow[code & 0xffff];
    }
}

}  // namespace hfmm
