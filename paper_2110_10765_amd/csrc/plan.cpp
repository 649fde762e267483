// Host-side basis planner: per-species configurations ("substates") and the
// A-block layout of the canonical order.  The many-body states themselves are
// written on the device (expand kernel); here only the configurations of each
// species are listed, which is tiny next to D.
#include <algorithm>
#include <functional>

#include "cib_internal.hpp"

namespace cib {

Orbs make_orbs(int nmax) {
  Orbs o;
  o.nmax = nmax;
  for (int n = 0; n <= nmax; ++n)
    for (int twoj = 1; twoj <= 2 * n + 1; twoj += 2)
      for (int twom = -twoj; twom <= twoj; twom += 2) {
        o.n.push_back(n);
        o.twoj.push_back(twoj);
        o.twom.push_back(twom);
      }
  o.n_orb = (int)o.n.size();
  o.words = (o.n_orb + 63) / 64;
  return o;
}

// Lowest summed quanta of N particles: orbitals are ordered by shell, so the
// first N orbitals fill the lowest shells.
int q_min(int N, const Orbs &o) {
  int q = 0;
  for (int k = 0; k < N; ++k) q += o.n[k];
  return q;
}

void validate_spec(const cib_basis_spec &s) {
  CIB_REQUIRE(s.n_species == 1 || s.n_species == 2, CIB_E_INVALID, "n_species must be 1 or 2");
  for (int sp = 0; sp < s.n_species; ++sp) {
    CIB_REQUIRE(s.nmax[sp] >= 0 && s.nmax[sp] <= 6, CIB_E_INVALID, "nmax must be in 0..6");
    int n_orb = (s.nmax[sp] + 1) * (s.nmax[sp] + 2) * (s.nmax[sp] + 3) / 3;
    CIB_REQUIRE(s.n_particles[sp] >= 1 && s.n_particles[sp] <= n_orb, CIB_E_INVALID,
                "particle number must be in 1..n_orb");
  }
  int N = s.n_particles[0] + (s.n_species == 2 ? s.n_particles[1] : 0);
  CIB_REQUIRE(((s.two_M - N) % 2 + 2) % 2 == 0, CIB_E_INVALID,
              "two_M must have the parity of the particle number");
}

// All N-particle configurations of one species with summed quanta <= qcap
// (qcap < 0: none), by recursion over orbitals in ascending order.
static void enum_configs(const Orbs &o, int N, int qcap, SubList &out) {
  uint64_t bits[kMaxWords] = {0, 0, 0};
  std::function<void(int, int, int, int)> rec = [&](int k0, int left, int m, int q) {
    if (left == 0) {
      for (int w = 0; w < kMaxWords; ++w) out.bits.push_back(bits[w]);
      out.m2.push_back(m);
      out.q.push_back(q);
      return;
    }
    for (int k = k0; k <= o.n_orb - left; ++k) {
      // orbitals are sorted by shell: every later particle costs >= o.n[k]
      if (qcap >= 0 && q + left * o.n[k] > qcap) break;
      bits[k >> 6] |= 1ull << (k & 63);
      rec(k + 1, left - 1, m + o.twom[k], q + o.n[k]);
      bits[k >> 6] &= ~(1ull << (k & 63));
    }
  };
  rec(0, N, 0, 0);
}

static bool int_less(const uint64_t *a, const uint64_t *b) {
  for (int w = kMaxWords - 1; w >= 0; --w)
    if (a[w] != b[w]) return a[w] < b[w];
  return false;
}

static void reorder(SubList &s, const std::vector<int> &idx) {
  SubList t;
  t.bits.resize(idx.size() * kMaxWords);
  t.m2.resize(idx.size());
  t.q.resize(idx.size());
  for (size_t i = 0; i < idx.size(); ++i) {
    std::memcpy(&t.bits[i * kMaxWords], &s.bits[(size_t)idx[i] * kMaxWords], sizeof(uint64_t) * kMaxWords);
    t.m2[i] = s.m2[idx[i]];
    t.q[i] = s.q[idx[i]];
  }
  s = std::move(t);
}

void make_plan(const cib_basis_spec &s, Plan &p) {
  validate_spec(s);
  p.spec = s;
  p.ns = s.n_species;
  p.oA = make_orbs(s.nmax[0]);
  p.oB = p.ns == 2 ? make_orbs(s.nmax[1]) : Orbs{};
  if (p.ns == 1) { p.oB.n_orb = 0; p.oB.words = 0; }
  p.WA = p.oA.words;
  p.WB = p.ns == 2 ? p.oB.words : 0;
  p.W = std::max(p.WA, std::max(p.WB, 1));
  const int NA = s.n_particles[0], NB = p.ns == 2 ? s.n_particles[1] : 0;
  const int qminA = q_min(NA, p.oA), qminB = p.ns == 2 ? q_min(NB, p.oB) : 0;
  p.qmax = s.cut >= 0 ? qminA + qminB + s.cut : -1;
  p.qminB = qminB;
  p.nlev = s.cut >= 0 ? s.cut + 1 : 1;

  SubList A, B;
  enum_configs(p.oA, NA, p.qmax >= 0 ? p.qmax - qminB : -1, A);
  if (p.ns == 2) {
    enum_configs(p.oB, NB, p.qmax >= 0 ? p.qmax - qminA : -1, B);
  } else {  // a single empty configuration stands in for the absent species
    for (int w = 0; w < kMaxWords; ++w) B.bits.push_back(0);
    B.m2.push_back(0);
    B.q.push_back(0);
  }
  // B: ascending (2M, Q, integer)
  {
    std::vector<int> idx(B.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) {
      if (B.m2[x] != B.m2[y]) return B.m2[x] < B.m2[y];
      if (B.q[x] != B.q[y]) return B.q[x] < B.q[y];
      return int_less(&B.bits[(size_t)x * kMaxWords], &B.bits[(size_t)y * kMaxWords]);
    });
    reorder(B, idx);
  }
  p.bseg_start.clear();
  p.bseg_m2.clear();
  p.b_seg.assign(B.size(), 0);
  for (size_t i = 0; i < B.size(); ++i) {
    if (i == 0 || B.m2[i] != B.m2[i - 1]) {
      p.bseg_start.push_back((int32_t)i);
      p.bseg_m2.push_back(B.m2[i]);
    }
    p.b_seg[i] = (int32_t)p.bseg_m2.size() - 1;
  }
  p.bseg_start.push_back((int32_t)B.size());
  CIB_REQUIRE(p.nseg() <= kMaxSeg, CIB_E_INVALID, "too many 2M segments");

  // A: ascending integer; keep configurations whose B list is non-empty
  std::vector<int> idx(A.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) {
    return int_less(&A.bits[(size_t)x * kMaxWords], &A.bits[(size_t)y * kMaxWords]);
  });
  std::vector<int> keep;
  p.a_len.clear();
  p.a_seg.clear();
  p.a_off.assign(1, 0);
  for (int k : idx) {
    int need = s.two_M - A.m2[k];
    auto it = std::lower_bound(p.bseg_m2.begin(), p.bseg_m2.end(), need);
    if (it == p.bseg_m2.end() || *it != need) continue;
    int g = (int)(it - p.bseg_m2.begin());
    int lo = p.bseg_start[g], hi = p.bseg_start[g + 1];
    int len = hi - lo;
    if (p.qmax >= 0) {  // prefix of entries with Q_B <= qmax - Q_A
      int cap = p.qmax - A.q[k];
      len = (int)(std::upper_bound(B.q.begin() + lo, B.q.begin() + hi, cap) - (B.q.begin() + lo));
    }
    if (len <= 0) continue;
    keep.push_back(k);
    p.a_len.push_back(len);
    p.a_seg.push_back(g);
    p.a_off.push_back(p.a_off.back() + len);
  }
  reorder(A, keep);
  p.A = std::move(A);
  p.B = std::move(B);
  p.D = p.a_off.back();
}

}  // namespace cib
