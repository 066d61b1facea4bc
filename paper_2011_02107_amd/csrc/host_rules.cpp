// Host-only rules of the DACP path (declarations and the statement of each rule in host_rules.h)
// and the host-only entry points of the C ABI: dacp_default_opts, dacp_plan, dacp_accept_rule,
// dacp_spacing_ratios.
#include "host_rules.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace dacp {
namespace rules {

double kpm_count(const std::vector<double> &mu, int64_t D, double a_r) {
  const int M = static_cast<int>(mu.size());
  const double q = M_PI / (M + 1);
  const double th = std::acos(a_r);
  double total = 0.0;
  for (int k = 0; k < M; ++k) {
    const double g = ((M - k + 1) * std::cos(q * k) + std::sin(q * k) / std::tan(q)) / (M + 1);
    if (k == 0) total += g * mu[0] * (M_PI - 2.0 * th) / M_PI;
    else total += 2.0 * g * mu[k] * (std::sin(k * (M_PI - th)) - std::sin(k * th)) / (k * M_PI);
  }
  return static_cast<double>(D) * total;
}

double window_for_count(const std::vector<double> &mu, int64_t D, double count) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (kpm_count(mu, D, mid) >= count) hi = mid;
    else lo = mid;
  }
  return hi;
}

std::vector<int64_t> sample_orders(double a_r, int n) {
  std::vector<int64_t> ks(n);
  for (int m = 1; m <= n; ++m) ks[m - 1] = 2 * static_cast<int64_t>(std::floor(m * M_PI / (2.0 * a_r)));
  return ks;
}

Plan make_plan(const dacp_opts &o, int64_t D, int N, double e_b, const std::vector<double> &mu, double window_ratio,
               int attempt) {
  Plan p;
  p.n_w = std::min(static_cast<double>(D), std::ceil(window_ratio * N));
  double a_r = (o.a > 0.0 && attempt == 0) ? o.a / e_b
                                           : window_for_count(mu.empty() ? std::vector<double>{1.0} : mu, D, p.n_w);
  if (o.a > 0.0 && attempt > 0) a_r = std::min(0.95, (o.a / e_b) * std::pow(1.5, attempt));
  p.a_r = std::min(a_r, 0.95);
  p.a = p.a_r * e_b;
  const double kfac = o.kfac > 0.0 ? o.kfac : 18.0;
  p.K = static_cast<int>(std::ceil(kfac / p.a_r));
  p.b = o.b;
  if (p.b <= 0) {
    p.b = 4;
    while (p.b < 64 && p.b * 16 <= p.n_w) p.b *= 2;
  }
  const double basis_ratio = o.basis_ratio > 0.0 ? o.basis_ratio : 1.5;
  p.n = std::max(1, static_cast<int>(std::ceil((basis_ratio * p.n_w / p.b - 1.0) / 2.0)));
  p.m = p.b * (2 * p.n + 1);
  return p;
}

std::vector<int> central_order(const std::vector<double> &theta) {
  std::vector<int> order(theta.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
    const double ai = std::fabs(theta[i]), aj = std::fabs(theta[j]);
    return ai < aj || (ai == aj && theta[i] < theta[j]);
  });
  return order;
}

AcceptResult accept_rule(const std::vector<double> &theta, const std::vector<int> &order, int n_sel,
                         const std::vector<double> &rnorm, double a, double tol) {
  const int r = static_cast<int>(theta.size());
  AcceptResult res;
  res.ok.assign(r, 0);
  res.ghost.assign(r, 0);
  res.est.assign(n_sel, INFINITY);
  // residual per Ritz value; NaN where it is not a candidate (not computed)
  std::vector<double> rho(r, NAN);
  std::vector<int> qpos(r, -1);
  for (int q = 0; q < n_sel; ++q) {
    const int j = order[q];
    rho[j] = rnorm[q];
    qpos[j] = q;
    if (!(rnorm[q] < a - std::fabs(theta[j]))) {  // also a NaN residual
      res.ghost[j] = 1;
      ++res.n_ghost;
    }
  }
  // non-ghost Ritz values in ascending order
  std::vector<int> g;
  g.reserve(r);
  for (int i = 0; i < r; ++i)
    if (!res.ghost[i]) g.push_back(i);
  const int ng = static_cast<int>(g.size());
  for (int p = 0; p < ng; ++p) {
    const int j = g[p];
    if (qpos[j] < 0) continue;  // not a candidate
    double est = rho[j];        // Weyl: a level within ||r||
    // every run g[lo..hi] containing p, at most kAcceptMaxCluster long, of candidates only
    for (int lo = p; lo >= 0 && p - lo < kAcceptMaxCluster && qpos[g[lo]] >= 0; --lo) {
      double r2 = 0.0, amax = 0.0;
      for (int i = lo; i < p; ++i) {
        r2 += rho[g[i]] * rho[g[i]];
        amax = std::max(amax, std::fabs(theta[g[i]]));
      }
      for (int hi = p; hi < ng && hi - lo < kAcceptMaxCluster && qpos[g[hi]] >= 0; ++hi) {
        r2 += rho[g[hi]] * rho[g[hi]];
        amax = std::max(amax, std::fabs(theta[g[hi]]));
        double delta = a - amax;
        if (lo > 0) {
          const int nb = g[lo - 1];
          const double rn = std::isnan(rho[nb]) ? 0.0 : rho[nb];
          delta = std::min(delta, theta[g[lo]] - theta[nb] - rn);
        }
        if (hi + 1 < ng) {
          const int nb = g[hi + 1];
          const double rn = std::isnan(rho[nb]) ? 0.0 : rho[nb];
          delta = std::min(delta, theta[nb] - theta[g[hi]] - rn);
        }
        if (delta > 0.0) est = std::min(est, r2 / delta);
      }
    }
    res.est[qpos[j]] = est;
    res.ok[j] = est <= tol;
  }
  for (int q = 0; q < n_sel && std::fabs(theta[order[q]]) <= a; ++q) {
    const int j = order[q];
    if (res.ghost[j] || !res.ok[j]) break;
    res.max_est = std::max(res.max_est, res.est[q]);
    res.core_idx.push_back(q);
  }
  return res;
}

int clusters_at_width(const double *eigs, int n, double tol, int b) {
  int count = 0, run = 1;
  for (int i = 1; i <= n; ++i) {
    if (i < n && eigs[i] - eigs[i - 1] <= 2.0 * tol) {
      ++run;
      continue;
    }
    if (run >= b && b >= 1 && n > 0) ++count;
    run = 1;
  }
  return count;
}

DcDeflation dc_deflate(const std::vector<double> &dv, const std::vector<double> &z, double rho, int lo) {
  const int n = static_cast<int>(dv.size());
  DcDeflation out;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return dv[a] < dv[b]; });
  out.ds.resize(n);
  out.zs.resize(n);
  out.rowid.resize(n);
  for (int i = 0; i < n; ++i) {
    out.ds[i] = dv[perm[i]];
    out.zs[i] = z[perm[i]];
    out.rowid[i] = lo + perm[i];
  }
  const double eps = 2.220446049250313e-16;
  double dmax = 0.0;
  for (double v : out.ds) dmax = std::max(dmax, std::fabs(v));
  const double tol = 8.0 * eps * std::max(dmax, rho);
  out.defl.assign(n, 0);
  int pj = -1;
  for (int j = 0; j < n; ++j) {
    if (rho * std::fabs(out.zs[j]) <= tol) {
      out.defl[j] = 1;
      continue;
    }
    if (pj >= 0) {
      const double s0 = out.zs[pj], c0 = out.zs[j];
      const double t = std::hypot(c0, s0);
      const double c = c0 / t, s = s0 / t;
      if (std::fabs((out.ds[j] - out.ds[pj]) * c * s) <= tol) {
        // rotate the pair so that z_pj = 0: rows pj' = c pj - s j, j' = s pj + c j
        out.rot_pq.push_back(out.rowid[pj]);
        out.rot_pq.push_back(out.rowid[j]);
        out.rot_cs.push_back(c);
        out.rot_cs.push_back(s);
        out.zs[j] = t;
        out.zs[pj] = 0.0;
        const double dp = out.ds[pj] * c * c + out.ds[j] * s * s;
        out.ds[j] = out.ds[pj] * s * s + out.ds[j] * c * c;
        out.ds[pj] = dp;
        out.defl[pj] = 1;
      }
    }
    pj = j;
  }
  for (int j = 0; j < n; ++j)
    if (!out.defl[j]) out.nd.push_back(j);
  return out;
}

std::vector<int64_t> anchor_orders(int64_t kn) {
  std::vector<int64_t> a;
  for (int64_t k : {int64_t(0), int64_t(1), int64_t(2), kn - 2, kn - 1, kn, kn + 1})
    if (k >= 0) a.push_back(k);
  std::sort(a.begin(), a.end());
  a.erase(std::unique(a.begin(), a.end()), a.end());
  return a;
}

MomentChain moment_chain(const std::vector<int64_t> &orders, const std::vector<int64_t> &anchors) {
  MomentChain out;
  const int64_t kn = orders.back();
  const int na = static_cast<int>(anchors.size()), npan = static_cast<int>(orders.size());
  struct Rule {
    int ai, q;
    int64_t k, other;  // the moment given; the one subtracted (-1: none)
  };
  std::unordered_map<int64_t, int> rule_of;  // order -> index into rules
  std::vector<Rule> rules;
  for (bool changed = true; changed;) {
    changed = false;
    for (int ai = 0; ai < na; ++ai)
      for (int q = 0; q < npan; ++q) {
        const int64_t sum = anchors[ai] + orders[q];
        const int64_t dif = anchors[ai] >= orders[q] ? anchors[ai] - orders[q] : orders[q] - anchors[ai];
        const bool hs = rule_of.count(sum) > 0, hd = rule_of.count(dif) > 0;
        int64_t k = -1, other = -1;
        if (sum == dif) {
          if (!hs) k = sum;
        } else if (hd && !hs) {
          k = sum;
          other = dif;
        } else if (hs && !hd) {
          k = dif;
          other = sum;
        }
        if (k < 0) continue;
        rule_of[k] = static_cast<int>(rules.size());
        rules.push_back({ai, q, k, other});
        changed = true;
      }
  }
  // the orders the assembly reads, and the rules they are derived from
  std::vector<char> needed(static_cast<size_t>(2 * kn) + 1, 0), used(rules.size(), 0);
  for (int64_t x : orders)
    for (int64_t y : orders) needed[x + y] = needed[x >= y ? x - y : y - x] = 1;
  for (int64_t k = 0; k <= 2 * kn; ++k) {
    if (!needed[k]) continue;
    auto it = rule_of.find(k);
    if (it == rule_of.end()) {
      out.missing = k;
      return out;
    }
    for (int r = it->second; r >= 0 && !used[r];) {
      used[r] = 1;
      r = rules[r].other < 0 ? -1 : rule_of.at(rules[r].other);
    }
  }
  std::vector<int> cidx(rules.size(), -1);
  int nc = 0;
  for (size_t r = 0; r < rules.size(); ++r) {
    if (!used[r]) continue;
    cidx[r] = nc++;
    out.table.push_back(rules[r].ai);
    out.table.push_back(rules[r].q);
    out.table.push_back(rules[r].other < 0 ? -1 : cidx[rule_of.at(rules[r].other)]);
    out.order.push_back(rules[r].k);
  }
  out.block_of.assign(needed.size(), -1);
  for (size_t k = 0; k < needed.size(); ++k)
    if (needed[k]) out.block_of[k] = cidx[rule_of.at(static_cast<int64_t>(k))];
  return out;
}

DcPlacement dc_place(std::vector<DcEntry> ents, int k) {
  std::stable_sort(ents.begin(), ents.end(), [](const DcEntry &a, const DcEntry &b) { return a.v < b.v; });
  DcPlacement out;
  const int n = static_cast<int>(ents.size());
  out.w.resize(n);
  out.dst_of_root.assign(k, -1);
  for (int t = 0; t < n; ++t) {
    if (ents[t].kind == 0) {
      out.src_defl.push_back(ents[t].idx);
      out.dst_defl.push_back(t);
    } else {
      out.dst_of_root[ents[t].idx] = t;
    }
    out.w[t] = ents[t].v;
  }
  return out;
}

}  // namespace rules
}  // namespace dacp

using dacp::rules::AcceptResult;
using dacp::rules::Plan;

extern "C" {

void dacp_default_opts(dacp_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->b = 0;
  o->group = 0;
  o->kfac = 18.0;
  o->window_ratio = 2.2;
  o->basis_ratio = 1.5;
  o->eps = 1e-12;
  o->tol_rel = 1e-10;
  o->lanczos_steps = 80;
  o->kpm_moments = 256;
  o->kpm_vectors = 8;
  o->e_bound = 0.0;
  o->a = 0.0;
  o->precision = DACP_F64;
  o->fp64_tail_frac = 0.2;
  o->seed = 0;
  o->max_retries = 1;
  o->sectors = 0;
}

dacp_status dacp_plan(int64_t D, int N, double e_bound, const double *mu, int n_mu, const dacp_opts *opts_in,
                      int attempt, double *fout, int *iout, int64_t *k_samples, int max_samples) {
  if (D < 1 || N < 1 || N > D || !(e_bound > 0.0) || attempt < 0 || !fout || !iout) return DACP_E_INVALID;
  dacp_opts o;
  if (opts_in) o = *opts_in;
  else dacp_default_opts(&o);
  if (!(o.a > 0.0) && (!mu || n_mu < 1)) return DACP_E_INVALID;
  std::vector<double> m;
  if (!(o.a > 0.0)) m.assign(mu, mu + n_mu);
  // the same widening as dacp_central_eigs applies before each retry
  double window_ratio = o.window_ratio > 0.0 ? o.window_ratio : 2.2;
  for (int i = 0; i < attempt; ++i) window_ratio *= 1.5;
  const Plan p = dacp::rules::make_plan(o, D, N, e_bound, m, window_ratio, attempt);
  fout[0] = p.n_w;
  fout[1] = p.a_r;
  fout[2] = p.a;
  iout[0] = p.K;
  iout[1] = p.b;
  iout[2] = p.n;
  iout[3] = p.m;
  if (k_samples && max_samples > 0) {
    const std::vector<int64_t> ks = dacp::rules::sample_orders(p.a_r, p.n);
    for (int i = 0; i < std::min(max_samples, p.n); ++i) k_samples[i] = ks[i];
  }
  return DACP_OK;
}

dacp_status dacp_accept_rule(int r, const double *theta, int n_sel, const double *rnorm, double a, double tol,
                             int *core_out, int *core_pos, double *est_out, int *n_ghost_out) {
  if (r < 0 || n_sel < 0 || n_sel > r || (r > 0 && !theta) || (n_sel > 0 && !rnorm) || !core_out || !(a > 0.0) ||
      !(tol >= 0.0))
    return DACP_E_INVALID;
  const std::vector<double> th(theta, theta + r);
  for (int i = 0; i + 1 < r; ++i)
    if (!(th[i + 1] >= th[i])) return DACP_E_INVALID;
  const std::vector<double> rn(rnorm, rnorm + n_sel);
  const AcceptResult res = dacp::rules::accept_rule(th, dacp::rules::central_order(th), n_sel, rn, a, tol);
  *core_out = static_cast<int>(res.core_idx.size());
  if (core_pos) std::copy(res.core_idx.begin(), res.core_idx.end(), core_pos);
  if (est_out) std::copy(res.est.begin(), res.est.end(), est_out);
  if (n_ghost_out) *n_ghost_out = res.n_ghost;
  return DACP_OK;
}

dacp_status dacp_spacing_ratios(const double *eigs, int n, double *r_out, double *mean_out) {
  if (!eigs || n < 3) return DACP_E_INVALID;
  for (int i = 0; i + 1 < n; ++i)
    if (!(eigs[i + 1] >= eigs[i])) return DACP_E_INVALID;  // also rejects NaN
  double sum = 0.0;
  int64_t cnt = 0;
  for (int i = 0; i + 2 < n; ++i) {
    const double s0 = eigs[i + 1] - eigs[i], s1 = eigs[i + 2] - eigs[i + 1];
    const double hi = std::max(s0, s1);
    const double r = hi > 0.0 ? std::min(s0, s1) / hi : NAN;
    if (r_out) r_out[i] = r;
    if (hi > 0.0) {
      sum += r;
      ++cnt;
    }
  }
  if (mean_out) *mean_out = cnt ? sum / static_cast<double>(cnt) : NAN;
  return DACP_OK;
}

}  // extern "C"
