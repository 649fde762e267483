// Host runtime: context, allocator cache, error reporting, interaction upload.
#include <algorithm>
#include <map>

#include "cib_internal.hpp"

namespace cib {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

DevInter cib_interaction_view(const cib_interaction &t);

// Pair layout of the blocked tables: blocks by 2M_pair ascending, pairs
// lexicographic inside a block.  pidx[a * n2 + b] = block << 16 | index.
struct PairLayout {
  std::vector<int32_t> pidx, vn;
  std::vector<int64_t> vbase;
  int64_t total = 0;
};

static PairLayout pair_layout(const Orbs &o1, const Orbs &o2, bool same) {
  std::map<int, std::vector<std::pair<int, int>>> blocks;
  for (int a = 0; a < o1.n_orb; ++a)
    for (int b = same ? a + 1 : 0; b < o2.n_orb; ++b) blocks[o1.twom[a] + o2.twom[b]].push_back({a, b});
  PairLayout L;
  L.pidx.assign((size_t)std::max(1, o1.n_orb * o2.n_orb), -1);
  int blk = 0;
  for (auto &kv : blocks) {
    auto &prs = kv.second;
    std::sort(prs.begin(), prs.end());
    CIB_REQUIRE(prs.size() < 65536, CIB_E_OVERFLOW, "pair block too large");
    for (size_t i = 0; i < prs.size(); ++i)
      L.pidx[(size_t)prs[i].first * o2.n_orb + prs[i].second] = (blk << 16) | (int32_t)i;
    L.vbase.push_back(L.total);
    L.vn.push_back((int32_t)prs.size());
    L.total += (int64_t)prs.size() * (int64_t)prs.size();
    ++blk;
  }
  if (L.vbase.empty()) { L.vbase.push_back(0); L.vn.push_back(0); }
  return L;
}

cib_interaction *upload_interaction(cib_ctx *ctx, const cib_basis &b, const cib_tables &t) {
  const Plan &p = b.plan;
  CIB_REQUIRE(t.eps[0] && t.v_same[0], CIB_E_INVALID, "tables: eps[0] and v_same[0] required");
  if (p.ns == 2)
    CIB_REQUIRE(t.eps[1] && t.v_same[1] && t.v_ab, CIB_E_INVALID,
                "tables: two species need eps[1], v_same[1] and v_ab");
  std::unique_ptr<cib_interaction> it(new cib_interaction);
  it->ctx = ctx;
  it->nA = p.oA.n_orb;
  it->nB = p.ns == 2 ? p.oB.n_orb : 0;
  hipStream_t s = ctx->stream;
  auto up_layout = [&](const PairLayout &L, const double *v, DBuf<int32_t> &pidx, DBuf<int32_t> &vn,
                       DBuf<int64_t> &vbase, DBuf<double> &dv) {
    pidx.reset(ctx, L.pidx.size());
    pidx.upload(L.pidx.data(), L.pidx.size(), s);
    vn.reset(ctx, L.vn.size());
    vn.upload(L.vn.data(), L.vn.size(), s);
    vbase.reset(ctx, L.vbase.size());
    vbase.upload(L.vbase.data(), L.vbase.size(), s);
    dv.reset(ctx, std::max<int64_t>(L.total, 1));
    dv.upload(v, (size_t)L.total, s);
  };
  it->epsA.reset(ctx, it->nA);
  it->epsA.upload(t.eps[0], it->nA, s);
  PairLayout LA = pair_layout(p.oA, p.oA, true);
  up_layout(LA, t.v_same[0], it->pidxA, it->vnA, it->vbaseA, it->vA);
  if (p.ns == 2) {
    it->epsB.reset(ctx, it->nB);
    it->epsB.upload(t.eps[1], it->nB, s);
    PairLayout LB = pair_layout(p.oB, p.oB, true);
    up_layout(LB, t.v_same[1], it->pidxB, it->vnB, it->vbaseB, it->vB);
    PairLayout LAB = pair_layout(p.oA, p.oB, false);
    up_layout(LAB, t.v_ab, it->pidxAB, it->vnAB, it->vbaseAB, it->vAB);
    it->dab.reset(ctx, (size_t)it->nA * it->nB);
    launch_dab(it->view(), it->dab.p, s);
  }
  // host arrays are copied before returning
  CIB_HIP(hipStreamSynchronize(s));
  return it.release();
}

}  // namespace cib

cib::DevInter cib_interaction::view() const {
  cib::DevInter v;
  v.nA = nA; v.nB = nB;
  v.epsA = epsA.p; v.epsB = epsB.p;
  v.pidxA = pidxA.p; v.vnA = vnA.p; v.vbaseA = vbaseA.p; v.vA = vA.p;
  v.pidxB = pidxB.p; v.vnB = vnB.p; v.vbaseB = vbaseB.p; v.vB = vB.p;
  v.pidxAB = pidxAB.p; v.vnAB = vnAB.p; v.vbaseAB = vbaseAB.p; v.vAB = vAB.p;
  v.dab = dab.p;
  return v;
}

// ------------------------------------------------------------------ context
static size_t round_up(size_t n) { return (n + 255) & ~(size_t)255; }

void *cib_ctx::alloc(size_t bytes) {
  bytes = round_up(std::max<size_t>(bytes, 256));
  void *p = nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (has_user) {
    p = user.alloc(bytes, user.user);
    CIB_REQUIRE(p, CIB_E_NOMEM, "allocator returned NULL");
  } else {
    auto it = cache.find(bytes);
    if (it != cache.end()) {
      p = it->second;
      cache.erase(it);
      cached -= (int64_t)bytes;
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {  // give the cache back and retry once
        (void)hipGetLastError();
        for (auto &kv : cache) (void)hipFree(kv.second);
        cache.clear();
        cached = 0;
        e = hipMalloc(&p, bytes);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw cib::Error(CIB_E_NOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
      }
    }
  }
  sizes[p] = bytes;
  live += (int64_t)bytes;
  peak = std::max(peak, live);
  return p;
}

void cib_ctx::free(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu);
  auto it = sizes.find(p);
  size_t bytes = it == sizes.end() ? 0 : it->second;
  if (it != sizes.end()) sizes.erase(it);
  live -= (int64_t)bytes;
  if (has_user) {
    user.free(p, user.user);
  } else {
    cache.emplace(bytes, p);
    cached += (int64_t)bytes;
  }
}

void cib_ctx::release_cache() {
  std::lock_guard<std::mutex> g(mu);
  for (auto &kv : cache) (void)hipFree(kv.second);
  cache.clear();
  cached = 0;
}

void *cib_ctx::pinned_buf(size_t bytes) {
  if (bytes > pinned_bytes) {
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    CIB_HIP(hipHostMalloc(&pinned, std::max<size_t>(bytes, 4096), hipHostMallocDefault));
    pinned_bytes = std::max<size_t>(bytes, 4096);
  }
  return pinned;
}
