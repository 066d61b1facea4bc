// Host-side harness of the library's host-only entry points and rules
// (paper_2011_02107_amd/csrc/host_rules.cpp): dacp_plan, dacp_accept_rule, dacp_spacing_ratios, the
// divide-and-conquer merge bookkeeping and the moment projection's derivation chain, on random and
// edge-case inputs.  Built with
// -fsanitize=address,undefined: any out-of-bounds access, use after free, overflow or other
// undefined behaviour aborts the run.  The checks here are invariants of each output (sizes,
// ranges, orderings, permutations); the values themselves are compared with the oracle elsewhere.
// Exit status 0 = every check held.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

#include "host_rules.h"

namespace {
int g_fail = 0;
void check(bool ok, const char *what, long a = 0) {
  if (!ok && g_fail++ < 20) std::fprintf(stderr, "FAIL: %s (%ld)\n", what, a);
}

void plans(std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int t = 0; t < 3000; ++t) {
    const int L = 1 + static_cast<int>(rng() % 24);
    const int64_t D = int64_t(1) << L;
    const int N = 1 + static_cast<int>(rng() % std::min<int64_t>(D, 6000));
    const double eb = 0.1 + 50.0 * u(rng);
    const int n_mu = 1 + static_cast<int>(rng() % 300);
    std::vector<double> mu(n_mu);
    mu[0] = 1.0;
    for (int k = 1; k < n_mu; ++k) mu[k] = (k % 2 ? 0.0 : std::exp(-0.01 * k) * (u(rng) - 0.3));
    dacp_opts o;
    dacp_default_opts(&o);
    if (t % 5 == 0) o.a = eb * (0.01 + 0.5 * u(rng));
    if (t % 7 == 0) o.b = 1 + static_cast<int>(rng() % 128);
    if (t % 11 == 0) o.kfac = 0.0;
    const int attempt = static_cast<int>(rng() % 4);
    double f[3];
    int it[4];
    const int maxs = static_cast<int>(rng() % 50);
    std::vector<int64_t> ks(std::max(1, maxs));
    const dacp_status st = dacp_plan(D, N, eb, mu.data(), n_mu, &o, attempt, f, it, ks.data(), maxs);
    check(st == DACP_OK, "dacp_plan on valid input", t);
    if (st != DACP_OK) continue;
    check(f[0] >= 1.0 && f[0] <= static_cast<double>(D), "plan: window count", t);
    check(f[1] > 0.0 && f[1] <= 0.95, "plan: a_r in (0, 0.95]", t);
    check(it[0] >= 1 && it[1] >= 1 && it[2] >= 1 && it[3] == it[1] * (2 * it[2] + 1), "plan: K, b, n, m", t);
    for (int i = 1; i < std::min(maxs, it[2]); ++i) check(ks[i] > ks[i - 1] && ks[i] % 2 == 0, "plan: orders", t);
  }
  double f[3];
  int it[4];
  check(dacp_plan(0, 1, 1.0, nullptr, 0, nullptr, 0, f, it, nullptr, 0) == DACP_E_INVALID, "plan: D = 0");
  check(dacp_plan(16, 17, 1.0, nullptr, 0, nullptr, 0, f, it, nullptr, 0) == DACP_E_INVALID, "plan: N > D");
  const double mu1 = 1.0;
  check(dacp_plan(16, 4, -1.0, &mu1, 1, nullptr, 0, f, it, nullptr, 0) == DACP_E_INVALID, "plan: E_b < 0");
  check(dacp_plan(16, 4, 1.0, nullptr, 0, nullptr, 0, f, it, nullptr, 0) == DACP_E_INVALID, "plan: no moments");
}

void acceptance(std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int t = 0; t < 3000; ++t) {
    const int r = static_cast<int>(rng() % 400);
    std::vector<double> th(r);
    for (double &x : th) x = 2.0 * u(rng) - 1.0;
    std::sort(th.begin(), th.end());
    if (r > 10 && t % 3 == 0)
      for (int i = 1; i < 5; ++i) th[r / 2 + i] = th[r / 2] + 1e-12 * i;  // a tight cluster
    if (r > 3 && t % 4 == 0) th[1] = th[0];                                // a repeated value
    const int n_sel = r ? static_cast<int>(rng() % (r + 1)) : 0;
    std::vector<double> rn(n_sel);
    for (double &x : rn) {
      const double v = u(rng);
      x = v < 0.03 ? NAN : (v < 0.08 ? 10.0 : std::pow(10.0, -14.0 + 11.0 * u(rng)));
    }
    const double a = 0.01 + u(rng), tol = std::pow(10.0, -12.0 + 5.0 * u(rng));
    int core = -1, ng = -1;
    std::vector<int> pos(std::max(1, n_sel), -7);
    std::vector<double> est(std::max(1, n_sel));
    const dacp_status st = dacp_accept_rule(r, th.data(), n_sel, rn.data(), a, tol, &core, pos.data(), est.data(), &ng);
    check(st == DACP_OK, "accept: valid input", t);
    if (st != DACP_OK) continue;
    check(core >= 0 && core <= n_sel && ng >= 0 && ng <= n_sel, "accept: counts", t);
    for (int i = 0; i < core; ++i) check(pos[i] == i, "accept: the core is a prefix of the candidates", t);
    for (int i = 0; i < core; ++i) check(est[pos[i]] <= tol, "accept: core estimates within tol", t);
    for (int q = 0; q < n_sel; ++q) check(!std::isnan(est[q]), "accept: estimate NaN", t);
  }
  int core;
  const double th2[2] = {0.2, 0.1}, rn1[1] = {1e-12};
  check(dacp_accept_rule(2, th2, 1, rn1, 0.5, 1e-10, &core, nullptr, nullptr, nullptr) == DACP_E_INVALID, "accept: unsorted");
  check(dacp_accept_rule(0, nullptr, 0, nullptr, 0.5, 1e-10, &core, nullptr, nullptr, nullptr) == DACP_OK && core == 0,
        "accept: empty");
  check(dacp_accept_rule(2, th2, 3, rn1, 0.5, 1e-10, &core, nullptr, nullptr, nullptr) == DACP_E_INVALID, "accept: n_sel > r");
}

void spacing(std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int t = 0; t < 500; ++t) {
    const int n = 3 + static_cast<int>(rng() % 200);
    std::vector<double> e(n);
    for (double &x : e) x = u(rng);
    if (t % 3 == 0)
      for (int i = 0; i < n; i += 3) e[i] = 0.5;
    std::sort(e.begin(), e.end());
    std::vector<double> r(n - 2);
    double mean = 0.0;
    check(dacp_spacing_ratios(e.data(), n, r.data(), &mean) == DACP_OK, "ratios: valid", t);
    for (double x : r) check(std::isnan(x) || (x >= 0.0 && x <= 1.0), "ratios: in [0, 1]", t);
  }
  const double bad[3] = {0.0, NAN, 1.0};
  check(dacp_spacing_ratios(bad, 3, nullptr, nullptr) == DACP_E_INVALID, "ratios: NaN");
  check(dacp_spacing_ratios(bad, 2, nullptr, nullptr) == DACP_E_INVALID, "ratios: n < 3");
}

void clusters(std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int t = 0; t < 2000; ++t) {
    const int n = static_cast<int>(rng() % 60);
    std::vector<double> e;
    while (static_cast<int>(e.size()) < n) {
      const double v = u(rng);
      const int rep = 1 + static_cast<int>(rng() % 6);
      for (int k = 0; k < rep && static_cast<int>(e.size()) < n; ++k) e.push_back(v + 1e-13 * k);
    }
    std::sort(e.begin(), e.end());
    const int b = 1 + static_cast<int>(rng() % 6);
    const double tol = 1e-12;
    // brute force: maximal runs with consecutive gaps <= 2 tol, counted when at least b long
    int want = 0;
    for (int i = 0; i < n;) {
      int j = i + 1;
      while (j < n && e[j] - e[j - 1] <= 2.0 * tol) ++j;
      if (j - i >= b) ++want;
      i = j;
    }
    check(dacp::rules::clusters_at_width(e.data(), n, tol, b) == want, "clusters_at_width", t);
  }
}

void deflation(std::mt19937_64 &rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int t = 0; t < 2000; ++t) {
    const int n = 1 + static_cast<int>(rng() % 300);
    const int lo = static_cast<int>(rng() % 1000);
    std::vector<double> dv(n), z(n);
    for (double &x : dv) x = (t % 4 == 0) ? std::floor(8.0 * u(rng)) : 2.0 * u(rng) - 1.0;  // repeats
    double zn = 0.0;
    for (double &x : z) {
      x = (u(rng) < 0.1) ? 0.0 : (u(rng) < 0.1 ? 1e-20 : 2.0 * u(rng) - 1.0);
      zn += x * x;
    }
    if (zn == 0.0) z[0] = zn = 1.0;
    for (double &x : z) x /= std::sqrt(zn);
    const double rho = 0.01 + u(rng);
    const dacp::rules::DcDeflation d = dacp::rules::dc_deflate(dv, z, rho, lo);
    check(static_cast<int>(d.ds.size()) == n && static_cast<int>(d.rowid.size()) == n, "deflate: sizes", t);
    std::vector<int> rows(d.rowid);
    std::sort(rows.begin(), rows.end());
    for (int i = 0; i < n; ++i) check(rows[i] == lo + i, "deflate: rows are a permutation of the block", t);
    check(d.rot_pq.size() == d.rot_cs.size() && d.rot_pq.size() <= 2 * static_cast<size_t>(n), "deflate: rotations", t);
    for (int v : d.rot_pq) check(v >= lo && v < lo + n, "deflate: rotation row in the block", t);
    for (size_t i = 0; i + 1 < d.rot_cs.size(); i += 2)
      check(std::fabs(d.rot_cs[i] * d.rot_cs[i] + d.rot_cs[i + 1] * d.rot_cs[i + 1] - 1.0) < 1e-12, "deflate: c^2+s^2", t);
    int nd = 0;
    for (int j = 0; j < n; ++j) nd += d.defl[j] ? 0 : 1;
    check(nd == static_cast<int>(d.nd.size()), "deflate: kept list", t);
    // placement: deflated entries by their rows, roots by index, in value order
    std::vector<dacp::rules::DcEntry> ents;
    for (int j = 0; j < n; ++j)
      if (d.defl[j]) ents.push_back({d.ds[j], 0, d.rowid[j]});
    for (int q = 0; q < nd; ++q) ents.push_back({d.ds[d.nd[q]] + 1e-3 * u(rng), 1, q});
    const dacp::rules::DcPlacement p = dacp::rules::dc_place(ents, nd);
    check(static_cast<int>(p.w.size()) == n, "place: size", t);
    for (int i = 0; i + 1 < n; ++i) check(p.w[i] <= p.w[i + 1], "place: ascending", t);
    std::vector<int> dst(p.dst_defl);
    dst.insert(dst.end(), p.dst_of_root.begin(), p.dst_of_root.end());
    std::sort(dst.begin(), dst.end());
    for (int i = 0; i < n; ++i) check(dst[i] == i, "place: destinations are a permutation", t);
  }
}
}  // namespace

// The moment projection's derivation chain: for uniform grids of every even step to 80 and up to 40
// sample pairs, every order x + y, |x - y| of two panel orders is reached; every kept rule's anchor
// and panel give the order it claims (as A + x or |A - x|), with its subtracted moment, when there
// is one, the other of the two and given by an earlier rule; orders not read get no rule.
void moment_chains() {
  for (int delta = 2; delta <= 80; delta += 2)
    for (int n = 1; n <= 40; ++n) {
      std::vector<int64_t> orders{0};
      for (int j = 1; j <= n; ++j) {
        orders.push_back(int64_t(j) * delta - 1);
        orders.push_back(int64_t(j) * delta);
      }
      const int64_t kn = orders.back();
      const std::vector<int64_t> anchors = dacp::rules::anchor_orders(kn);
      check(std::is_sorted(anchors.begin(), anchors.end()) && anchors.front() == 0 && anchors.back() == kn + 1,
            "anchor orders", n);
      const dacp::rules::MomentChain ch = dacp::rules::moment_chain(orders, anchors);
      check(ch.missing < 0, "moment chain: an order is not reached", delta * 100 + n);
      const int nc = static_cast<int>(ch.order.size());
      check(ch.table.size() == static_cast<size_t>(3 * nc), "moment chain: table size", nc);
      check(ch.block_of.size() == static_cast<size_t>(2 * kn + 1), "moment chain: block map size", n);
      for (int c = 0; c < nc; ++c) {
        const int ai = ch.table[3 * c], q = ch.table[3 * c + 1], o = ch.table[3 * c + 2];
        if (ai < 0 || ai >= static_cast<int>(anchors.size()) || q < 0 || q >= static_cast<int>(orders.size()) ||
            o >= c) {
          check(false, "moment chain: rule out of range", c);
          continue;
        }
        const int64_t sum = anchors[ai] + orders[q];
        const int64_t dif = anchors[ai] >= orders[q] ? anchors[ai] - orders[q] : orders[q] - anchors[ai];
        const int64_t k = ch.order[c];
        if (o < 0) {
          check(sum == dif && k == sum, "moment chain: direct rule", c);
        } else {
          const int64_t ko = ch.order[o];
          check((k == sum && ko == dif) || (k == dif && ko == sum), "moment chain: derived rule", c);
        }
      }
      std::vector<char> needed(static_cast<size_t>(2 * kn) + 1, 0);
      for (int64_t x : orders)
        for (int64_t y : orders) needed[x + y] = needed[x >= y ? x - y : y - x] = 1;
      for (int64_t k = 0; k <= 2 * kn; ++k) {
        const int blk = ch.block_of[k];
        if (needed[k])
          check(blk >= 0 && blk < nc && ch.order[blk] == k, "moment chain: needed order's block", k);
        else
          check(blk == -1, "moment chain: unneeded order has a block", k);
      }
    }
}

int main() {
  std::mt19937_64 rng(20111);
  plans(rng);
  acceptance(rng);
  spacing(rng);
  clusters(rng);
  deflation(rng);
  moment_chains();
  std::printf("host rules harness: %d failures\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}
