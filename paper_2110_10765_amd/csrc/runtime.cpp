// Host runtime: context, allocator cache, error reporting, interaction upload.
#include <algorithm>
#include <exception>
#include <map>

#include "cib_internal.hpp"

namespace cib {

static thread_local std::string g_last_error;

static thread_local UnwindFence *t_fence = nullptr;

UnwindFence::UnwindFence(hipStream_t s) : s_(s), prev_(t_fence), depth_(std::uncaught_exceptions()) {
  t_fence = this;
}

UnwindFence::~UnwindFence() { t_fence = prev_; }

void UnwindFence::wait_if_unwinding() {
  UnwindFence *f = t_fence;
  if (!f || f->waited_ || std::uncaught_exceptions() <= f->depth_) return;
  (void)hipStreamSynchronize(f->s_);  // the error being thrown is the one reported
  f->waited_ = true;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

DevInter cib_interaction_view(const cib_interaction &t);

// Pair layout of the blocked tables: blocks by 2M_pair ascending, pairs
// lexicographic inside a block.  pidx[a * n2 + b] = block << 16 | index.
struct PairLayout {
  std::vector<int32_t> pidx;   // per ordered pair: block << 16 | index, -1 if not stored
  std::vector<int64_t> prow;   // per ordered pair: offset of its row in the blocked table
  int64_t total = 0;
};

static PairLayout pair_layout(const Orbs &o1, const Orbs &o2, bool same) {
  std::map<int, std::vector<std::pair<int, int>>> blocks;
  for (int a = 0; a < o1.n_orb; ++a)
    for (int b = same ? a + 1 : 0; b < o2.n_orb; ++b) blocks[o1.twom[a] + o2.twom[b]].push_back({a, b});
  PairLayout L;
  const size_t npair = (size_t)std::max(1, o1.n_orb * o2.n_orb);
  L.pidx.assign(npair, -1);
  L.prow.assign(npair, 0);
  int blk = 0;
  for (auto &kv : blocks) {
    auto &prs = kv.second;
    std::sort(prs.begin(), prs.end());
    CIB_REQUIRE(prs.size() < 65536, CIB_E_OVERFLOW, "pair block too large");
    for (size_t i = 0; i < prs.size(); ++i) {
      const size_t q = (size_t)prs[i].first * o2.n_orb + prs[i].second;
      L.pidx[q] = (blk << 16) | (int32_t)i;
      L.prow[q] = L.total + (int64_t)i * (int64_t)prs.size();
    }
    L.total += (int64_t)prs.size() * (int64_t)prs.size();
    ++blk;
  }
  return L;
}

// Transition layout of V^AB: A transitions (a <- c, a == c included) grouped
// by 2m_a - 2m_c, B transitions (b <- d) by 2m_b - 2m_d, both groups in
// lexicographic order.  Block for difference k: the A group k against the B
// group -k (the only B transitions that conserve the total 2M), row-major.
struct TransLayout {
  std::vector<int32_t> atr, btr;     // (a << 16 | c) and (b << 16 | d), group by group
  std::vector<int32_t> arb, bcol;    // per ordered orbital pair: row base, column index
  std::vector<VtBlock> blocks;
  int64_t total = 0;
};

static TransLayout trans_layout(const Orbs &oa, const Orbs &ob) {
  std::map<int, std::vector<int32_t>> ga, gb;
  for (int a = 0; a < oa.n_orb; ++a)
    for (int c = 0; c < oa.n_orb; ++c) ga[oa.twom[a] - oa.twom[c]].push_back((a << 16) | c);
  for (int b = 0; b < ob.n_orb; ++b)
    for (int d = 0; d < ob.n_orb; ++d) gb[ob.twom[b] - ob.twom[d]].push_back((b << 16) | d);
  TransLayout T;
  T.arb.assign((size_t)oa.n_orb * oa.n_orb, 0);
  T.bcol.assign((size_t)ob.n_orb * ob.n_orb, 0);
  std::map<int, int32_t> boff;
  for (auto &kv : gb) {
    boff[kv.first] = (int32_t)T.btr.size();
    for (size_t j = 0; j < kv.second.size(); ++j) {
      const int32_t e = kv.second[j];
      T.bcol[(size_t)(e >> 16) * ob.n_orb + (e & 0xffff)] = (int32_t)j;
      T.btr.push_back(e);
    }
  }
  for (auto &kv : ga) {
    const auto bit = gb.find(-kv.first);
    const int32_t nb = bit == gb.end() ? 0 : (int32_t)bit->second.size();
    VtBlock B{T.total, (int32_t)T.atr.size(), (int32_t)kv.second.size(), nb ? boff[-kv.first] : 0, nb};
    for (size_t i = 0; i < kv.second.size(); ++i) {
      const int32_t e = kv.second[i];
      T.arb[(size_t)(e >> 16) * oa.n_orb + (e & 0xffff)] = (int32_t)(T.total + (int64_t)i * nb);
      T.atr.push_back(e);
    }
    T.total += (int64_t)B.na * nb;
    // (the row passes address it with 32-bit byte offsets)
    CIB_REQUIRE(T.total < (int64_t(1) << 29), CIB_E_OVERFLOW, "transition table exceeds 2^29 entries");
    if (nb) T.blocks.push_back(B);
  }
  return T;
}

const char *const kKernelNames[K_NKERN] = {"screens", "row_count", "scan",
                                           "row_fill", "spmm_sym", "gram", "rayleigh_ritz", "update",
                                           "state_count", "apply_free"};

static hipEvent_t take_event(cib_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  // timing only: no system-scope fence (no cache writeback and invalidate
  // at every record)
  CIB_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

KTimer::KTimer(cib_ctx *c, int kernel, hipStream_t st) : ctx(c), k(kernel), s(st) {
  if (!ctx || !ctx->profiling) return;
  std::lock_guard<std::mutex> g(ctx->mu);
  a = take_event(ctx);
  b = take_event(ctx);
  CIB_HIP(hipEventRecord(a, s));
}

KTimer::~KTimer() {
  if (!a) return;
  std::lock_guard<std::mutex> g(ctx->mu);
  if (hipEventRecord(b, s) == hipSuccess) ctx->marks.push_back({k, a, b});
}

// Resolve completed marks into per-kernel totals (synchronises their events).
void profile_collect(cib_ctx *c) {
  std::lock_guard<std::mutex> g(c->mu);
  for (auto &m : c->marks) {
    float ms = 0.f;
    if (hipEventSynchronize(m.b) == hipSuccess && hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      auto &t = c->kernel_totals[m.kernel];
      t.first += 1;
      t.second += ms * 1e-3;
    }
    c->event_pool.push_back(m.a);
    c->event_pool.push_back(m.b);
  }
  c->marks.clear();
}

void profile_add(cib_ctx *c, int kernel, double seconds) {
  if (!c || !c->profiling) return;
  std::lock_guard<std::mutex> g(c->mu);
  auto &t = c->kernel_totals[kernel];
  t.first += 1;
  t.second += seconds;
}

size_t profile_marks(cib_ctx *c) {
  std::lock_guard<std::mutex> g(c->mu);
  return c->marks.size();
}

void profile_drop_marks(cib_ctx *c, size_t from) {
  std::lock_guard<std::mutex> g(c->mu);
  for (size_t k = from; k < c->marks.size(); ++k) {
    // the events may still be pending: wait before they go back to the pool
    (void)hipEventSynchronize(c->marks[k].b);
    c->event_pool.push_back(c->marks[k].a);
    c->event_pool.push_back(c->marks[k].b);
  }
  if (from < c->marks.size()) c->marks.resize(from);
}

cib_interaction *upload_interaction(cib_ctx *ctx, const cib_basis &b, const cib_tables &t,
                                    hipStream_t s) {
  const Plan &p = b.plan;
  CIB_REQUIRE(t.eps[0] && t.v_same[0], CIB_E_INVALID, "tables: eps[0] and v_same[0] required");
  if (p.ns == 2)
    CIB_REQUIRE(t.eps[1] && t.v_same[1] && t.v_ab, CIB_E_INVALID,
                "tables: two species need eps[1], v_same[1] and v_ab");
  UnwindFence fence(s);
  std::unique_ptr<cib_interaction> it(new cib_interaction);
  it->ctx = ctx;
  it->nA = p.oA.n_orb;
  it->nB = p.ns == 2 ? p.oB.n_orb : 0;
  auto up_layout = [&](const PairLayout &L, const double *v, DBuf<int32_t> &pidx, DBuf<int64_t> &prow,
                       DBuf<double> &dv) {
    pidx.reset(ctx, L.pidx.size());
    pidx.upload(L.pidx.data(), L.pidx.size(), s);
    prow.reset(ctx, L.prow.size());
    prow.upload(L.prow.data(), L.prow.size(), s);
    dv.reset(ctx, std::max<int64_t>(L.total, 1));
    dv.upload(v, (size_t)L.total, s);
  };
  it->epsA.reset(ctx, it->nA);
  it->epsA.upload(t.eps[0], it->nA, s);
  PairLayout LA = pair_layout(p.oA, p.oA, true);
  up_layout(LA, t.v_same[0], it->pidxA, it->prowA, it->vA);
  if (p.ns == 2) {
    it->epsB.reset(ctx, it->nB);
    it->epsB.upload(t.eps[1], it->nB, s);
    PairLayout LB = pair_layout(p.oB, p.oB, true);
    up_layout(LB, t.v_same[1], it->pidxB, it->prowB, it->vB);
    PairLayout LAB = pair_layout(p.oA, p.oB, false);
    up_layout(LAB, t.v_ab, it->pidxAB, it->prowAB, it->vAB);
    it->dab.reset(ctx, (size_t)it->nA * it->nB);
    launch_dab(it->view(), it->dab.p, s);
    // V^AB re-laid out by orbital transitions (one access per matrix entry)
    TransLayout T = trans_layout(p.oA, p.oB);
    DBuf<int32_t> atr(ctx, std::max<size_t>(T.atr.size(), 1)), btr(ctx, std::max<size_t>(T.btr.size(), 1));
    DBuf<VtBlock> blk(ctx, std::max<size_t>(T.blocks.size(), 1));
    atr.upload(T.atr.data(), T.atr.size(), s);
    btr.upload(T.btr.data(), T.btr.size(), s);
    blk.upload(T.blocks.data(), T.blocks.size(), s);
    it->arb.reset(ctx, T.arb.size());
    it->arb.upload(T.arb.data(), T.arb.size(), s);
    it->bcol.reset(ctx, T.bcol.size());
    it->bcol.upload(T.bcol.data(), T.bcol.size(), s);
    it->vt.reset(ctx, (size_t)std::max<int64_t>(T.total, 1));
    launch_build_vt(it->view(), blk.p, (int)T.blocks.size(), atr.p, btr.p, T.total, it->vt.p, s);
    CIB_HIP(hipStreamSynchronize(s));
    // the blocked pair tables are not read after this point
    it->vAB.release();
    it->pidxAB.release();
    it->prowAB.release();
  }
  // host arrays are copied before returning
  CIB_HIP(hipStreamSynchronize(s));
  return it.release();
}


// Device bytes the context allocator takes for a request of n bytes.
size_t dev_bytes(size_t n) { return n ? (std::max<size_t>(n, 256) + 255) & ~(size_t)255 : 0; }

// Peak device bytes of upload_interaction (every table, the transition
// staging and the blocked cross tables it frees at the end).
size_t interaction_device_bytes(const Plan &p) {
  auto lay = [](const PairLayout &L) {
    return dev_bytes(L.pidx.size() * 4) + dev_bytes(L.prow.size() * 8) +
           dev_bytes((size_t)std::max<int64_t>(L.total, 1) * 8);
  };
  size_t n = dev_bytes((size_t)p.oA.n_orb * 8) + lay(pair_layout(p.oA, p.oA, true));
  if (p.ns == 2) {
    const TransLayout T = trans_layout(p.oA, p.oB);
    n += dev_bytes((size_t)p.oB.n_orb * 8) + lay(pair_layout(p.oB, p.oB, true)) +
         lay(pair_layout(p.oA, p.oB, false)) + dev_bytes((size_t)p.oA.n_orb * p.oB.n_orb * 8) +
         dev_bytes(std::max<size_t>(T.atr.size(), 1) * 4) + dev_bytes(std::max<size_t>(T.btr.size(), 1) * 4) +
         dev_bytes(std::max<size_t>(T.blocks.size(), 1) * sizeof(VtBlock)) + dev_bytes(T.arb.size() * 4) +
         dev_bytes(T.bcol.size() * 4) + dev_bytes((size_t)std::max<int64_t>(T.total, 1) * 8);
  }
  return n;
}

// Device bytes of a basis made from plan p (make_basis).
size_t basis_device_bytes(const Plan &p) {
  const size_t W = p.W, nA = p.nA(), nB = p.nB(), D = p.D;
  auto i32 = [](size_t n) { return dev_bytes(std::max<size_t>(n, 1) * 4); };
  return dev_bytes(W * nA * 8) + dev_bytes(W * nB * 8) + i32(p.A.m2.size()) + i32(p.A.q.size()) +
         i32(p.a_len.size()) + i32(p.a_seg.size()) + i32(p.B.m2.size()) + i32(p.B.q.size()) +
         i32(p.b_seg.size()) + i32(p.bseg_start.size()) + dev_bytes(p.a_off.size() * 8) + 3 * dev_bytes(D * 4) +
         dev_bytes((size_t)(p.WA + p.WB) * D * 8);
}

cib_basis *make_basis(cib_ctx *ctx, const cib_basis_spec &spec, hipStream_t s) {
  Plan p;
  make_plan(spec, p);
  return make_basis(ctx, std::move(p), s);
}

cib_basis *make_basis(cib_ctx *ctx, Plan &&plan, hipStream_t s) {
  UnwindFence fence(s);
  std::unique_ptr<cib_basis> b(new cib_basis);
  b->ctx = ctx;
  b->plan = std::move(plan);
  const Plan &p = b->plan;
  CIB_REQUIRE(p.D > 0, CIB_E_EMPTY_BASIS, "the spec admits no state");
  CIB_REQUIRE(p.D < (int64_t(1) << 31), CIB_E_OVERFLOW, "basis dimension exceeds 2^31-1");
  const int W = p.W, nA = p.nA(), nB = p.nB();
  std::vector<uint64_t> soa((size_t)W * nA);
  for (int k = 0; k < nA; ++k)
    for (int w = 0; w < W; ++w) soa[(size_t)w * nA + k] = p.A.bits[(size_t)k * kMaxWords + w];
  b->a_bits.reset(ctx, soa.size());
  b->a_bits.upload(soa.data(), soa.size(), s);
  std::vector<uint64_t> sob((size_t)W * nB);
  for (int k = 0; k < nB; ++k)
    for (int w = 0; w < W; ++w) sob[(size_t)w * nB + k] = p.B.bits[(size_t)k * kMaxWords + w];
  b->b_bits.reset(ctx, sob.size());
  b->b_bits.upload(sob.data(), sob.size(), s);
  auto up32 = [&](DBuf<int32_t> &d, const std::vector<int32_t> &h) {
    d.reset(ctx, std::max<size_t>(h.size(), 1));
    d.upload(h.data(), h.size(), s);
  };
  up32(b->a_m2, p.A.m2);
  up32(b->a_q, p.A.q);
  up32(b->a_len, p.a_len);
  up32(b->a_seg, p.a_seg);
  up32(b->b_m2, p.B.m2);
  up32(b->b_q, p.B.q);
  up32(b->b_seg, p.b_seg);
  up32(b->bseg_start, p.bseg_start);
  b->a_off.reset(ctx, p.a_off.size());
  b->a_off.upload(p.a_off.data(), p.a_off.size(), s);
  b->row_a.reset(ctx, p.D);
  b->row_p.reset(ctx, p.D);
  b->row_b.reset(ctx, p.D);
  b->words.reset(ctx, (size_t)(p.WA + p.WB) * p.D);
  launch_expand_basis(*b, s);
  CIB_HIP(hipStreamSynchronize(s));  // host staging vectors go out of scope
  return b.release();
}

}  // namespace cib

cib::DevInter cib_interaction::view() const {
  cib::DevInter v;
  v.nA = nA; v.nB = nB;
  v.epsA = epsA.p; v.epsB = epsB.p;
  v.pidxA = pidxA.p; v.prowA = prowA.p; v.vA = vA.p;
  v.pidxB = pidxB.p; v.prowB = prowB.p; v.vB = vB.p;
  v.pidxAB = pidxAB.p; v.prowAB = prowAB.p; v.vAB = vAB.p;
  v.dab = dab.p;
  v.vt = vt.p; v.arb = arb.p; v.bcol = bcol.p;
  return v;
}

// ------------------------------------------------------------------ context
static size_t round_up(size_t n) { return (n + 255) & ~(size_t)255; }

// A user allocator hook may run HIP calls of its own (torch's caching
// allocator does, also on the library's worker threads): the device it
// leaves current is put back, and an error it leaves on this thread is its
// own and is discarded, so that the library's next launch check does not
// report it.
template <typename F>
static void *call_hook(F &&f) {
  int dev = -1;
  const bool have = hipGetDevice(&dev) == hipSuccess;
  void *r = f();
  int now = -1;
  if (have && hipGetDevice(&now) == hipSuccess && now != dev) (void)hipSetDevice(dev);
  (void)hipGetLastError();
  return r;
}

void *cib_ctx::alloc(size_t bytes) {
  bytes = round_up(std::max<size_t>(bytes, 256));
  void *p = nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (has_user) {
    p = call_hook([&] { return user.alloc(bytes, user.user); });
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
    call_hook([&] {
      user.free(p, user.user);
      return (void *)nullptr;
    });
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
