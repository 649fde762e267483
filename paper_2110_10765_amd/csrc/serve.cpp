// Continuous-batching serving loop (cib_serve).
//
// Host threads share one context:
//   builders (four, one stream each) take requests in arrival order once they
//            have arrived and a slot is free, build the basis and the
//            interaction tables, run the counting passes of the H build, then
//            wait until the request's whole device footprint (H, LOBPCG state,
//            build scratch) fits the HBM budget, fill H and hand the request to
//            the solver;
//   solver   keeps every admitted request's H and LOBPCG state resident and,
//            each step, enqueues one stage for every active request
//            (initialisation for new ones, one LOBPCG iteration for the rest)
//            (a new solve starts on its own stream); the iterating requests
//            run each stage of their iteration as one launch over all of them
//            (their workgroups in one grid; the Rayleigh-Ritz step one
//            workgroup per request).  It then waits once, reads
//            every status block from pinned memory, and retires converged
//            requests (releasing their memory and budget).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "cib_internal.hpp"

namespace cib {

namespace {

using clk = std::chrono::steady_clock;

struct Job {
  int idx = 0;
  const cib_request *req = nullptr;
  cib_result *res = nullptr;
  std::unique_ptr<cib_basis> basis;
  std::unique_ptr<cib_interaction> inter;
  std::unique_ptr<cib_matrix> H;
  LobpcgRun *lp = nullptr;
  size_t reserved = 0;
  int stream = 0;
  bool started = false;
  double *status = nullptr;  // pinned host slot
  ~Job() {
    if (lp) lobpcg_destroy(lp);
  }
};

struct Shared {
  std::mutex mu;
  std::condition_variable cv;
  size_t budget = 0, in_use = 0;
  int active = 0, max_active = 64;
  std::deque<Job *> ready;
  bool builder_done = false;
  bool cancelled = false;
};

}  // namespace

// A request gives way (frees what it holds and starts again later) when its
// build needs more of the budget than is free: waiting while holding memory
// could deadlock the builders.
struct GiveWay {};

cib_status serve_run(cib_ctx *ctx, const cib_request *reqs, int n, const cib_serve_opts &o,
                     cib_result *results) {
  const auto t0 = clk::now();
  auto now = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
  Shared sh;
  sh.max_active = o.max_active > 0 ? o.max_active : 64;
  const int nstreams = o.n_streams > 0 ? o.n_streams : 8;
  if (o.hbm_budget_bytes) {
    sh.budget = o.hbm_budget_bytes;
  } else {
    size_t fr = 0, tot = 0;
    CIB_HIP(hipMemGetInfo(&fr, &tot));
    sh.budget = (size_t)(0.9 * (double)fr);
  }
  const double deadline = o.deadline_s > 0 ? o.deadline_s : 1e300;

  for (int i = 0; i < n; ++i) {
    cib_result &r = results[i];
    std::memset(&r, 0, sizeof(r));
    r.id = reqs[i].id;
    r.status = CIB_E_CANCELLED;
    r.t_arrive = o.realtime ? reqs[i].arrival_s : 0.0;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

  // several builder threads (one stream each): the builds of small requests
  // are bound by launches and host waits, so they overlap well
  const int nbuild = 4;
  std::vector<hipStream_t> streams(nstreams + 1 + nbuild, nullptr);
  for (auto &st : streams) CIB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipStream_t gstream = streams[nstreams];   // batched Rayleigh-Ritz steps
  double *pinned = nullptr;
  CIB_HIP(hipHostMalloc((void **)&pinned, sizeof(double) * kStatusLen * (size_t)sh.max_active,
                        hipHostMallocDefault));
  GroupRunner runner(ctx);   // grouped iterations (arguments staged in pinned memory)
  std::vector<int> free_slots;
  for (int k = sh.max_active - 1; k >= 0; --k) free_slots.push_back(k);
  std::string builder_error;
  cib_status builder_status = CIB_OK;

  // ------------------------------------------------------------ builder threads
  std::atomic<int> next_k{0};
  int builders_left = nbuild;
  auto builder_fn = [&](int bt) {
    int dev = ctx->device;
    (void)hipSetDevice(dev);
    hipStream_t bstream = streams[nstreams + 1 + bt];
    for (;;) {
      const int k = next_k.fetch_add(1);
      if (k >= n) break;
      const int i = order[k];
      const cib_request &q = reqs[i];
      cib_result &res = results[i];
      if (o.realtime) {
        const double wait = q.arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      }
      {
        std::unique_lock<std::mutex> lk(sh.mu);
        sh.cv.wait(lk, [&] { return sh.active < sh.max_active || sh.cancelled; });
        if (sh.cancelled) break;
        ++sh.active;
      }
      if (now() > deadline) {
        std::lock_guard<std::mutex> lk(sh.mu);
        --sh.active;
        sh.cv.notify_all();
        continue;  // stays CIB_E_CANCELLED
      }
      res.t_admit = now();
      std::unique_ptr<Job> job(new Job);
      job->idx = i;
      job->req = &q;
      job->res = &res;
      cib_status st = CIB_OK;
      // the budget covers everything a request allocates: basis and tables,
      // the build's scratch, H and the solver state.  Each allocation group is reserved (exact bytes) before it is
      // made; only the first reservation waits, with nothing held.
      auto unreserve = [&](size_t bytes) {
        std::lock_guard<std::mutex> lk(sh.mu);
        sh.in_use -= bytes;
        job->reserved -= bytes;
        sh.cv.notify_all();
      };
      try {
        CIB_REQUIRE(q.tables, CIB_E_INVALID, "request without tables");
        CIB_REQUIRE(q.solve.x0 == nullptr, CIB_E_INVALID, "serving requests cannot pass x0");
        CIB_REQUIRE(q.solve.precond == nullptr, CIB_E_INVALID, "serving requests cannot pass a preconditioner");
        CIB_REQUIRE(q.solve.nev >= 1 && q.solve.nev <= 16, CIB_E_INVALID, "nev must be in 1..16");
        Plan plan;
        make_plan(q.basis, plan);
        CIB_REQUIRE(plan.D > 0, CIB_E_EMPTY_BASIS, "the spec admits no state");
        res.dim = plan.D;
        CIB_REQUIRE(3 * (int64_t)q.solve.block <= res.dim, CIB_E_INVALID, "need 3 * block <= D");
        const size_t basis_b = basis_device_bytes(plan), inter_b = interaction_device_bytes(plan);
        size_t known = basis_b + inter_b;   // grows as a build learns its sizes
        for (;;) {
          CIB_REQUIRE(known <= sh.budget, CIB_E_NOMEM, "request footprint exceeds the HBM budget");
          {
            std::unique_lock<std::mutex> lk(sh.mu);
            sh.cv.wait(lk, [&] { return sh.in_use + known <= sh.budget || sh.cancelled; });
            CIB_REQUIRE(!sh.cancelled, CIB_E_CANCELLED, "cancelled");
            sh.in_use += known;
            job->reserved = known;
          }
          size_t stages = 0, scratch = 0;
          try {
            job->basis.reset(make_basis(ctx, Plan(plan), bstream));
            job->inter.reset(upload_interaction(ctx, *job->basis, *q.tables, bstream));
            job->H.reset(new cib_matrix);
            job->H->ctx = ctx;
            // stages 0, 1: scratch freed when the build returns; 2: the
            // stored entries (with them, the solver state they will need)
            const BuildReserve reserve = [&](int stage, size_t bytes) {
              if (stage < 2) scratch += bytes;
              if (stage == 2) bytes += lobpcg_bytes(plan.D, q.solve.block, q.dtype);
              stages += bytes;
              const size_t want = basis_b + inter_b + stages;
              known = std::max(known, want);
              if (job->reserved >= want) return;
              CIB_REQUIRE(want <= sh.budget, CIB_E_NOMEM, "request footprint exceeds the HBM budget");
              std::lock_guard<std::mutex> lk(sh.mu);
              const size_t more = want - job->reserved;
              if (sh.in_use + more > sh.budget) throw GiveWay{};
              sh.in_use += more;
              job->reserved += more;
            };
            build_matrix(ctx, *job->basis, *job->inter, q.dtype, *job->H, bstream, reserve);
          } catch (const GiveWay &) {
            // everything built so far is released (its stream drained first)
            // and the request starts again once its whole known footprint fits
            job->H.reset();
            job->inter.reset();
            job->basis.reset();
            unreserve(job->reserved);
            continue;
          }
          res.nnz_half = job->H->nnz;
          job->inter.reset();            // tables are no longer needed once H is built
          unreserve(inter_b + scratch);  // the build's scratch is gone too
          break;
        }
      } catch (const Error &e) {
        st = e.code;
        if (st == CIB_E_DEVICE) {
          std::lock_guard<std::mutex> lk(sh.mu);
          builder_error = e.what();
          builder_status = st;
        }
      } catch (const std::exception &e) {
        st = CIB_E_DEVICE;
        std::lock_guard<std::mutex> lk(sh.mu);
        builder_error = e.what();
        builder_status = st;
      }
      if (st != CIB_OK) {
        res.status = st;
        res.t_done = now();
        std::lock_guard<std::mutex> lk(sh.mu);
        sh.in_use -= job->reserved;
        --sh.active;
        sh.cv.notify_all();
        if (builder_status != CIB_OK) { sh.cancelled = true; break; }
        continue;
      }
      std::lock_guard<std::mutex> lk(sh.mu);
      sh.ready.push_back(job.release());
      sh.cv.notify_all();
    }
    std::lock_guard<std::mutex> lk(sh.mu);
    if (--builders_left == 0) sh.builder_done = true;
    sh.cv.notify_all();
  };
  std::vector<std::thread> builders;
  for (int bt = 0; bt < nbuild; ++bt) builders.emplace_back(builder_fn, bt);

  // ------------------------------------------------------------ solver loop
  std::vector<Job *> active;
  int next_stream = 0;
  cib_status loop_status = CIB_OK;
  std::string loop_error;
  try {
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(sh.mu);
        if (active.empty())
          sh.cv.wait(lk, [&] { return !sh.ready.empty() || sh.builder_done; });
        while (!sh.ready.empty()) {
          Job *j = sh.ready.front();
          sh.ready.pop_front();
          j->stream = next_stream;
          next_stream = (next_stream + 1) % nstreams;
          j->status = pinned + (size_t)free_slots.back() * kStatusLen;
          free_slots.pop_back();
          active.push_back(j);
        }
        if (active.empty() && sh.builder_done) break;
      }
      if (now() > deadline) break;
      // enqueue one stage per active request: a new solve starts on its own
      // stream; the others run one iteration together, every stage of it one
      // launch over all of them (a solve the grouped SpMM cannot take
      // iterates on its own stream)
      std::vector<LobpcgRun *> g_runs;
      std::vector<IterPlan> g_plans;
      std::vector<Job *> g_jobs;
      std::vector<Job *> failed;
      for (Job *j : active) {
        hipStream_t s = streams[j->stream];
        if (!j->started) {
          cib_lobpcg_opts lo = j->req->solve;
          try {
            j->lp = lobpcg_create(ctx, *j->H, lo, s);
          } catch (const Error &e) {
            if (e.code != CIB_E_NOMEM) throw;
            failed.push_back(j);   // this request alone fails; the others go on
            continue;
          }
          lobpcg_start(j->lp);
          j->started = true;
          lobpcg_copy_status(j->lp, j->status);
          continue;
        }
        IterPlan p;
        if (lobpcg_plan_iteration(j->lp, p)) {
          g_runs.push_back(j->lp);
          g_plans.push_back(p);
          g_jobs.push_back(j);
        } else {
          lobpcg_iterate(j->lp);
          lobpcg_copy_status(j->lp, j->status);
        }
      }
      if (!g_runs.empty()) {
        runner.run(g_runs, g_plans, gstream);
        for (size_t q = 0; q < g_jobs.size(); ++q)
          CIB_HIP(hipMemcpyAsync(g_jobs[q]->status, g_plans[q].status, sizeof(double) * kStatusLen,
                                 hipMemcpyDeviceToHost, gstream));
      }
      for (int k = 0; k < nstreams; ++k) CIB_HIP(hipStreamSynchronize(streams[k]));
      CIB_HIP(hipStreamSynchronize(gstream));
      // retire (and release the requests whose solver state did not fit)
      auto release = [&](Job *j) {
        free_slots.push_back((int)((j->status - pinned) / kStatusLen));
        const size_t rel = j->reserved;
        delete j;
        std::lock_guard<std::mutex> lk(sh.mu);
        sh.in_use -= rel;
        --sh.active;
        sh.cv.notify_all();
      };
      for (Job *j : failed) {
        j->res->status = CIB_E_NOMEM;
        j->res->t_done = now();
        active.erase(std::find(active.begin(), active.end(), j));
        release(j);
      }
      std::vector<Job *> keep;
      for (Job *j : active) {
        const int nev = j->req->solve.nev;
        const int conv = (int)j->status[0];
        const int it = lobpcg_iters(j->lp);
        const bool done = conv >= nev || it >= j->req->solve.max_iter;
        if (!done) { keep.push_back(j); continue; }
        cib_result &r = *j->res;
        r.status = conv >= nev ? CIB_OK : CIB_E_NOT_CONVERGED;
        r.iters = it;
        for (int k = 0; k < nev; ++k) {
          r.resid[k] = j->status[1 + k];
          r.evals[k] = j->status[1 + kMaxBlock + k];
        }
        r.t_done = now();
        release(j);
      }
      active.swap(keep);
    }
  } catch (const Error &e) {
    loop_status = e.code;
    loop_error = e.what();
  } catch (const std::exception &e) {
    loop_status = CIB_E_DEVICE;
    loop_error = e.what();
  }
  {
    std::lock_guard<std::mutex> lk(sh.mu);
    sh.cancelled = true;
    sh.cv.notify_all();
  }
  for (auto &t : builders) t.join();
  for (auto &st : streams) (void)hipStreamSynchronize(st);
  for (Job *j : active) delete j;
  for (Job *j : sh.ready) delete j;
  for (auto &st : streams) (void)hipStreamDestroy(st);

  (void)hipHostFree(pinned);
  if (loop_status != CIB_OK) throw Error(loop_status, loop_error);
  if (builder_status != CIB_OK) throw Error(builder_status, builder_error);
  return CIB_OK;
}

}  // namespace cib
