// Serving loop: admission by device-memory budget, assembly of newly admitted
// requests on their own contexts and streams, and an engine that advances
// every live request by one Krylov step per round with the operator products
// of all requests in grouped launches.  Included at the end of api.cpp (it
// uses the solver building blocks of that translation unit).

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ServeRecord {
  uint64_t ticket = 0;
  // copied inputs
  std::vector<std::vector<double>> verts;
  std::vector<std::vector<int32_t>> tris;
  std::vector<pmchwt_complex> eps;
  double k_ext = 0;
  int nrhs = 0;
  std::vector<double> dirs;
  std::vector<pmchwt_complex> pols;
  pmchwt_assembly_opts oA{}, oP{};
  int precond = 0;
  pmchwt_solver_opts so{};
  int64_t est = 0, N = 0;
  // state (guarded by the server mutex)
  int status = PMCHWT_PENDING;
  bool cancel = false;
  int skipped = 0;  // times a later request was admitted ahead of this one at the head
  double t_submit = 0, t_admit = 0, t_done = 0;
  pmchwt_solve_stats stats{};
  std::vector<pmchwt_complex> currents;
  std::vector<double> sext, ssca;
};

// Device-memory estimate of one request (upper bound of what its context
// allocates: operators, slot-row slabs of the assembly, near-field P, mass
// matrices and their inverses, Krylov space and solve buffers).
int64_t serve_estimate(const ServeRecord& r) {
  double Etot = 0, Fmax = 0, Emax = 0, mass = 0, Aint = 0, slab = 0;
  for (auto& t : r.tris) {
    const double F = double(t.size() / 3), E = 1.5 * F;
    Etot += E;
    Fmax = std::max(Fmax, F);
    Emax = std::max(Emax, E);
  }
  const double elt = r.oA.precision == PMCHWT_FP64 ? 16.0 : 8.0;
  for (auto& t : r.tris) {
    const double E = 1.5 * double(t.size() / 3), F = double(t.size() / 3);
    Aint += 2.0 * E * double(padld(int64_t(E))) * elt;
    mass += 4.0 * E * E * 8.0 + 2.0 * E * double(ldmass(int64_t(E))) * 8.0 + 4.0 * E * 128.0 * 8.0;
    slab = std::max(slab, std::min(SLAB_BUDGET, F * 3.0 * 2.0 * (elt / 2.0) * 2.0 * (Etot + E)));
  }
  const double A = 2.0 * Etot * double(padld(int64_t(Etot))) * elt + Aint;
  const double nnz = std::isfinite(r.oP.chi) && r.oP.chi >= 0 ? Etot * std::min(Etot, 800.0) : Etot * Etot;
  const double P = nnz * (4.0 * 16.0 + 12.0);
  const double N = 2.0 * Etot, nr = r.nrhs, rho = r.so.restart;
  const double kry = (rho + 6.0) * nr * N * 16.0 * 2.0 + 10.0 * nr * N * 16.0 + 2.0 * 4.0 * nr * 2.0 * (Etot + 32) * 4.0;
  const double tables = 6.0 * Etot * 400.0;
  // FP64 copy of A for the refinement residuals of MIXED requests with many
  // right-hand sides (full rows of every operator, FP64 slot-row slabs)
  double a64 = 0.0;
  if (r.oA.precision == PMCHWT_MIXED && r.so.ir_max > 0 && r.nrhs >= FREE_MAX_RHS) {
    a64 = 2.0 * Etot * double(padld(int64_t(Etot))) * 16.0;
    for (auto& t : r.tris) {
      const double E = 1.5 * double(t.size() / 3);
      a64 += 2.0 * E * double(padld(int64_t(E))) * 16.0;
    }
    a64 += slab;
  }
  return int64_t(1.15 * (A + slab + P + mass + kry + tables + a64) + 64.0e6);
}

// One admitted request: its context, solve buffers and the staged solve
// (main GMRES, then iterative refinement as in pmchwt_solve).
struct ServeRun {
  enum Stage { MAIN, IR_CHECK, IR_SOLVE, FINISHED };
  std::shared_ptr<ServeRecord> rec;
  pmchwt_ctx* c = nullptr;
  int nrhs = 0;
  int64_t vs = 0;
  size_t nd = 0;
  DBuf b, bt, x, s1, s2, d, r, sA;
  std::unique_ptr<GmresRun> g;
  Stage st = MAIN;
  int ir = 0, it_max = 0, restarts = 0;
  std::vector<int> conv;
  std::vector<double> relres;
  std::unique_ptr<PinnedBuf> hn;
  hipEvent_t ev = nullptr;
  double t0 = 0;
  bool grouped = false;  // this step's operator product is in the grouped launches

  ~ServeRun() {
    g.reset();
    if (ev) (void)hipEventDestroy(ev);
    b = DBuf();
    bt = DBuf();
    x = DBuf();
    s1 = DBuf();
    s2 = DBuf();
    d = DBuf();
    r = DBuf();
    sA = DBuf();
    g_inc = DBuf();
    c_inc = DBuf();
    hn.reset();
    if (c) pmchwt_destroy(c);
  }

  // MIXED operators with refinement: FP64 residuals r = g/2 - A^i (c_inc +
  // x) - A^e x (one matrix-free FP64 product each), as in pmchwt_solve
  bool fp64_ir = false;
  DBuf g_inc, c_inc;

  void init() {
    const pmchwt_solver_opts& o = rec->so;
    vs = vlen(c);
    nd = size_t(2 * vs * nrhs);
    b = dalloc_c<double>(c, nd);
    bt = dalloc_c<double>(c, nd);
    x = dalloc_c<double>(c, nd);
    s1 = dalloc_c<double>(c, nd);
    s2 = dalloc_c<double>(c, nd);
    d = dalloc_c<double>(c, nd);
    r = dalloc_c<double>(c, nd);
    sA = dalloc_c<double>(c, nd);
    hn.reset(new PinnedBuf(16 * size_t(nrhs)));
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    t0 = now_ms();
    fp64_ir = c->precA == PMCHWT_MIXED && o.ir_max > 0;
    build_rhs(c, rec->dirs.data(), rec->pols.data(), nrhs, b.as<double>(), false, fp64_ir ? &g_inc : nullptr,
              fp64_ir ? &c_inc : nullptr);
    c->calls_A = 0;
    c->calls_P = 0;
    apply_Ptilde(c, b.as<double>(), bt.as<double>(), s1.as<double>(), s2.as<double>(), nrhs);
    g.reset(new GmresRun(c, bt.as<double>(), x.as<double>(), nrhs, o.tol, o.restart, o.max_iter));
    g->start();
    conv.assign(nrhs, 0);
    relres.assign(nrhs, 1.0);
    advance_after_gmres();
  }

  // after the GMRES run of the current stage has no more steps
  void advance_after_gmres() {
    if (g->phase != GmresRun::DONE) return;
    int mi = 0;
    for (int q = 0; q < nrhs; ++q) {
      mi = std::max(mi, g->out.iters[q]);
      conv[q] = g->out.converged[q];
      relres[q] = g->out.relres[q];
      if (st == MAIN) restarts = std::max(restarts, g->out.restarts[q]);
    }
    it_max += mi;
    if (st == IR_SOLVE) {
      launch_axpby(x.as<double>(), d.as<double>(), vs, int(vs), nrhs, 1.0, 1.0, c->stream);
      ++ir;
    }
    g.reset();
    st = rec->so.ir_max > 0 ? IR_CHECK : FINISHED;
  }

  bool stepping() const { return st != FINISHED; }

  // operator-product input and output of this step (A x into out)
  void a_io(const double*& in, double*& out) const {
    if (st == IR_CHECK) {
      in = x.as<double>();
      out = r.as<double>();
    } else {
      in = g->op_in();
      out = c->precond == PMCHWT_P_I ? g->op_out() : sA.as<double>();
    }
  }

  // the rest of the step's operator application, enqueued on the run's stream
  void post_A() {
    if (st == IR_CHECK) {  // r = b - A x, s1 = Ptilde r, |s1|, |bt|
      if (fp64_ir)  // r held A^i (c_inc + x) + A^e x
        launch_axpby(r.as<double>(), g_inc.as<double>(), vs, int(vs), nrhs, -1.0, 0.5, c->stream);
      else
        launch_axpby(r.as<double>(), b.as<double>(), vs, int(vs), nrhs, -1.0, 1.0, c->stream);
      apply_Ptilde(c, r.as<double>(), s1.as<double>(), s2.as<double>(), d.as<double>(), nrhs);
      double* dn = g_norm_scratch();
      launch_norms(s1.as<double>(), vs, int(vs), nrhs, dn, c->stream);
      launch_norms(bt.as<double>(), vs, int(vs), nrhs, dn + nrhs, c->stream);
      HIPCHK(hipMemcpyAsync(hn->p, dn, 16 * size_t(nrhs), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipEventRecord(ev, c->stream));
    } else if (c->precond != PMCHWT_P_I) {
      apply_Ptilde(c, sA.as<double>(), g->op_out(), g->s2, g->s3, nrhs);
    }
  }
  double* g_norm_scratch() { return s2.as<double>(); }  // 2 nrhs doubles, free during the check

  void stage1() {
    if (st == MAIN || st == IR_SOLVE) g->stage1();
  }
  void stage2() {
    if (st == MAIN || st == IR_SOLVE) {
      g->stage2();
      return;
    }
    if (st != IR_CHECK) return;
    HIPCHK(hipEventSynchronize(ev));
    const double* h = static_cast<const double*>(hn->p);
    bool ok = true;
    std::vector<double> tq(nrhs);
    for (int q = 0; q < nrhs; ++q) {
      const bool okq = h[q] <= rec->so.tol * h[nrhs + q];
      ok &= okq;
      conv[q] = okq ? 1 : 0;
      relres[q] = h[nrhs + q] > 0 ? h[q] / h[nrhs + q] : 0.0;
      tq[q] = correction_tol(rec->so.tol, h[q], h[nrhs + q]);
    }
    if (ok || ir == rec->so.ir_max) {
      st = FINISHED;
      return;
    }
    HIPCHK(hipMemcpyAsync(r.p, s1.p, nd * 8, hipMemcpyDeviceToDevice, c->stream));
    g.reset(new GmresRun(c, r.as<double>(), d.as<double>(), nrhs, rec->so.tol, rec->so.restart, rec->so.max_iter,
                         tq.data()));
    st = IR_SOLVE;
    g->start();
    advance_after_gmres();
  }
  void stage3() {
    if (st == MAIN || st == IR_SOLVE) {
      g->stage3();
      advance_after_gmres();
    }
  }

  // currents, cross sections and statistics into the record (synchronous)
  void finish() {
    std::vector<double> h(nd);
    HIPCHK(hipMemcpyAsync(h.data(), x.p, nd * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    rec->currents.resize(size_t(nrhs) * 2 * c->E_tot);
    to_api(c, h, nrhs, rec->currents.data());
    rec->sext.assign(nrhs, 0.0);
    rec->ssca.assign(nrhs, 0.0);
    const int rc = pmchwt_cross_sections(c, rec->currents.data(), nrhs, rec->dirs.data(), rec->pols.data(),
                                         rec->sext.data(), rec->ssca.data());
    if (rc != PMCHWT_OK) throw Fail{rc, c->err};
    bool ok = true;
    double worst = 0;
    for (int q = 0; q < nrhs; ++q) {
      ok &= bool(conv[q]);
      worst = std::max(worst, relres[q]);
    }
    pmchwt_solve_stats& s = rec->stats;
    s.iterations = it_max;
    s.converged = ok;
    s.matvecs = c->calls_A * A_matvecs(c) + c->calls_P * P_matvecs(c);
    s.rel_residual = worst;
    s.ir_steps = ir;
    s.restarts = restarts;
    s.ms_solve = now_ms() - t0;
  }
};

}  // namespace

struct pmchwt_server {
  int device = 0;
  size_t budget = 0;
  int max_live = 1;
  std::mutex m;
  std::condition_variable cv_admit, cv_engine, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::shared_ptr<ServeRecord>> recs;
  std::deque<std::shared_ptr<ServeRecord>> pending;
  std::vector<std::unique_ptr<ServeRun>> ready;
  int live_count = 0;  // admitted (assembling or in the engine)
  int64_t used = 0;
  pmchwt_server_stats st{};
  std::thread admit_thr, engine_thr, reap_thr;
  hipStream_t es = nullptr;  // engine stream (grouped launches)
  struct JobStage {
    std::unique_ptr<PinnedBuf> h;
    DBuf d;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
  } jst[2];
  int jcur = 0;
  // finished or cancelled runs: copied out, their contexts destroyed and their
  // budget released by the reaper thread (hipFree waits for the whole
  // device, which the engine must not)
  std::deque<std::unique_ptr<ServeRun>> reap;
  std::condition_variable cv_reap;
  std::string err;

  void admit_loop();
  void engine_loop();
  void reap_loop();
  void round(std::vector<std::unique_ptr<ServeRun>>& live);
  void complete(const std::shared_ptr<ServeRecord>& rec, int status);
  int pick_admissible();
};

namespace {

// grouped operator launches of one round: jobs by (interior?, precision, nr)
template <typename M>
struct JobLists {
  std::vector<GemvJob<M>> j[2][3];  // [exterior, interior][nr 4, 2, 1]
  int blocks[2][3] = {{0, 0, 0}, {0, 0, 0}};
  void add(int part, const M* S, const M* C, int64_t ld, int rows, int cols, double kr, double ki, const double* xD,
           const double* xN, double* yD, double* yN, int nrhs, int64_t vs) {
    for (int r0 = 0; r0 < nrhs;) {
      const int left = nrhs - r0, nr = left >= 4 ? 4 : (left >= 2 ? 2 : 1), k = nr == 4 ? 0 : (nr == 2 ? 1 : 2);
      GemvJob<M> g{S, C, ld, rows, cols, kr, ki, xD + 2 * int64_t(r0) * vs, xN + 2 * int64_t(r0) * vs,
                   yD + 2 * int64_t(r0) * vs, yN + 2 * int64_t(r0) * vs, vs, blocks[part][k]};
      blocks[part][k] += gemv_blocks<M>(rows, nr);
      j[part][k].push_back(g);
      r0 += nr;
    }
  }
};

}  // namespace

void pmchwt_server::complete(const std::shared_ptr<ServeRecord>& rec, int status) {
  std::lock_guard<std::mutex> lk(m);
  rec->status = status;
  rec->t_done = now_ms();
  if (status == PMCHWT_OK || status == PMCHWT_ERR_NOT_CONVERGED)
    st.completed++;
  else
    st.failed++;
  cv_done.notify_all();
}

// Index of the pending request to admit next, or -1 (server mutex held).
// First fit in submission order: a later request that fits the remaining
// budget may pass a head request that does not, until the head has been
// passed HEAD_PASS_LIMIT times; from then on only the head is admitted, so a
// large request is never starved.
constexpr int HEAD_PASS_LIMIT = 8;
int pmchwt_server::pick_admissible() {
  if (live_count >= max_live || pending.empty()) return -1;
  const int64_t room = int64_t(budget) - used;
  if (pending.front()->est <= room) return 0;
  if (pending.front()->skipped >= HEAD_PASS_LIMIT) return -1;
  for (size_t i = 1; i < pending.size(); ++i)
    if (!pending[i]->cancel && pending[i]->est <= room) return int(i);
  return -1;
}

void pmchwt_server::reap_loop() {
  (void)hipSetDevice(device);
  while (true) {
    std::unique_ptr<ServeRun> up;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_reap.wait(lk, [&] { return stop || !reap.empty(); });
      if (reap.empty()) return;  // stopping with nothing left
      up = std::move(reap.front());
      reap.pop_front();
    }
    std::shared_ptr<ServeRecord> rec = up->rec;
    bool cancel;
    {
      std::lock_guard<std::mutex> lk(m);
      cancel = rec->cancel;
    }
    int status = PMCHWT_ERR_CANCELLED;
    if (!cancel) {
      status = guarded(up->c, [&]() -> int {
        up->finish();
        return rec->stats.converged ? PMCHWT_OK : PMCHWT_ERR_NOT_CONVERGED;
      });
    }
    const int64_t est = rec->est;
    up.reset();  // frees the request's device memory
    {
      std::lock_guard<std::mutex> lk(m);
      live_count--;
      used -= est;
    }
    complete(rec, status);
    cv_admit.notify_all();
  }
}

void pmchwt_server::admit_loop() {
  (void)hipSetDevice(device);
  while (true) {
    std::shared_ptr<ServeRecord> rec;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_admit.wait(lk, [&] {
        if (stop) return true;
        for (size_t i = 0; i < pending.size();) {  // drop cancelled ones
          if (!pending[i]->cancel) {
            ++i;
            continue;
          }
          auto p = pending[i];
          pending.erase(pending.begin() + i);
          p->status = PMCHWT_ERR_CANCELLED;
          p->t_done = now_ms();
          st.failed++;
          cv_done.notify_all();
        }
        return pick_admissible() >= 0;
      });
      if (stop) return;
      const int pick = pick_admissible();
      rec = pending[size_t(pick)];
      pending.erase(pending.begin() + pick);
      if (pick > 0) pending.front()->skipped++;
      rec->status = PMCHWT_RUNNING;
      rec->t_admit = now_ms();
      live_count++;
      used += rec->est;
    }
    std::unique_ptr<ServeRun> run(new ServeRun());
    run->rec = rec;
    run->nrhs = rec->nrhs;
    int rc = pmchwt_create(&run->c, device, nullptr);
    if (rc == PMCHWT_OK) run->c->comb_ok = false;
    for (size_t q = 0; rc == PMCHWT_OK && q < rec->verts.size(); ++q)
      rc = pmchwt_add_scatterer(run->c, rec->verts[q].data(), int32_t(rec->verts[q].size() / 3), rec->tris[q].data(),
                                int32_t(rec->tris[q].size() / 3), rec->eps[q], nullptr);
    if (rc == PMCHWT_OK) rc = pmchwt_set_wavenumber(run->c, rec->k_ext);
    if (rc == PMCHWT_OK) rc = pmchwt_assemble(run->c, &rec->oA, &rec->oP, pmchwt_precond(rec->precond));
    if (rc == PMCHWT_OK) rc = guarded(run->c, [&]() -> int {
      run->init();
      return PMCHWT_OK;
    });
    if (rc != PMCHWT_OK) {
      run.reset();
      {
        std::lock_guard<std::mutex> lk(m);
        live_count--;
        used -= rec->est;
      }
      complete(rec, rc);
      cv_admit.notify_all();
      continue;
    }
    std::lock_guard<std::mutex> lk(m);
    ready.push_back(std::move(run));
    cv_engine.notify_all();
  }
}

void pmchwt_server::round(std::vector<std::unique_ptr<ServeRun>>& live) {
  JobLists<float> jf;
  JobLists<double> jd;
  // 1. the operator products: zero the outputs on each run's stream, then either
  //    the run's own matrix-core product or jobs of the grouped launches
  for (auto& up : live) {
    ServeRun& R = *up;
    pmchwt_ctx* c = R.c;
    const double* in;
    double* out;
    R.a_io(in, out);
    const int64_t E = c->E_tot, vs = R.vs;
    R.grouped = !(c->precA == PMCHWT_MIXED && R.nrhs >= MFMA_MIN_RHS);
    if (R.st == ServeRun::IR_CHECK && R.fp64_ir) {  // FP64 refinement residual on the run's stream
      R.grouped = false;
      // interior input c_inc + x in d (free until the check's own scratch use)
      HIPCHK(hipMemcpyAsync(R.d.p, R.c_inc.p, R.nd * 8, hipMemcpyDeviceToDevice, c->stream));
      launch_axpby(R.d.as<double>(), in, vs, int(vs), R.nrhs, 1.0, 1.0, c->stream);
      apply_A_resid(c, in, R.d.as<double>(), out, R.nrhs);
      continue;
    }
    if (!R.grouped) {
      apply_A(c, in, out, R.nrhs);
      continue;
    }
    c->calls_A += 1;
    launch_zero(out, 2 * vs * R.nrhs, c->stream);
    HIPCHK(hipEventRecord(R.ev, c->stream));
    HIPCHK(hipStreamWaitEvent(es, R.ev, 0));
    if (c->precA == PMCHWT_FP64) {
      jd.add(0, c->Se.as<double>(), c->Ce.as<double>(), c->ldE, int(E), int(E), c->k_ext, 0.0, in, in + 2 * E, out,
             out + 2 * E, R.nrhs, vs);
      for (size_t m = 0; m < c->sc.size(); ++m) {
        const Scat& s = c->sc[m];
        const int64_t o = s.edge_off;
        jd.add(1, c->Si[m].as<double>(), c->Ci[m].as<double>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
               s.k.imag(), in + 2 * o, in + 2 * (E + o), out + 2 * o, out + 2 * (E + o), R.nrhs, vs);
      }
    } else {
      jf.add(0, c->Se.as<float>(), c->Ce.as<float>(), c->ldE, int(E), int(E), c->k_ext, 0.0, in, in + 2 * E, out,
             out + 2 * E, R.nrhs, vs);
      for (size_t m = 0; m < c->sc.size(); ++m) {
        const Scat& s = c->sc[m];
        const int64_t o = s.edge_off;
        jf.add(1, c->Si[m].as<float>(), c->Ci[m].as<float>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
               s.k.imag(), in + 2 * o, in + 2 * (E + o), out + 2 * o, out + 2 * (E + o), R.nrhs, vs);
      }
    }
  }
  // 2. grouped launches on the engine stream: all exterior products, then all
  //    interior ones (a run's interior rows add to rows its exterior product
  //    wrote, in the order of a launch of that run alone)
  size_t bytes = 0;
  for (int part = 0; part < 2; ++part)
    for (int k = 0; k < 3; ++k)
      bytes += jf.j[part][k].size() * sizeof(GemvJob<float>) + jd.j[part][k].size() * sizeof(GemvJob<double>);
  if (bytes > 0) {
    // the job table goes through one of two staging pairs (pinned host and
    // device), used in alternate rounds and grown geometrically: a pair is
    // rewritten only after the launches of its previous round have finished,
    // which its event tells without stopping the engine stream
    JobStage& J = jst[jcur];
    jcur ^= 1;
    if (J.used) HIPCHK(hipEventSynchronize(J.done));
    if (J.cap < bytes) {
      const size_t cap = std::max<size_t>({bytes, 2 * J.cap, size_t(64) << 10});
      J.h.reset(new PinnedBuf(cap));
      J.d = dalloc<char>(cap);
      J.cap = cap;
    }
    DBuf& dj = J.d;
    char* hp = static_cast<char*>(J.h->p);
    size_t off = 0;
    struct L {
      size_t off;
      int n, nr, blocks, part, prec;
    };
    std::vector<L> ls;
    const int NR[3] = {4, 2, 1};
    for (int part = 0; part < 2; ++part)
      for (int k = 0; k < 3; ++k) {
        if (!jf.j[part][k].empty()) {
          std::memcpy(hp + off, jf.j[part][k].data(), jf.j[part][k].size() * sizeof(GemvJob<float>));
          ls.push_back({off, int(jf.j[part][k].size()), NR[k], jf.blocks[part][k], part, 0});
          off += jf.j[part][k].size() * sizeof(GemvJob<float>);
        }
        if (!jd.j[part][k].empty()) {
          std::memcpy(hp + off, jd.j[part][k].data(), jd.j[part][k].size() * sizeof(GemvJob<double>));
          ls.push_back({off, int(jd.j[part][k].size()), NR[k], jd.blocks[part][k], part, 1});
          off += jd.j[part][k].size() * sizeof(GemvJob<double>);
        }
      }
    HIPCHK(hipMemcpyAsync(dj.p, J.h->p, bytes, hipMemcpyHostToDevice, es));
    for (int part = 0; part < 2; ++part)
      for (const L& l : ls) {
        if (l.part != part) continue;
        if (l.prec == 0)
          launch_gemv_pmchwt_grouped<float>(reinterpret_cast<const GemvJob<float>*>(dj.as<char>() + l.off), l.n,
                                            l.nr, l.blocks, es);
        else
          launch_gemv_pmchwt_grouped<double>(reinterpret_cast<const GemvJob<double>*>(dj.as<char>() + l.off), l.n,
                                             l.nr, l.blocks, es);
        HIPCHK(hipGetLastError());
        std::lock_guard<std::mutex> lk(m);
        st.grouped_launches++;
        st.grouped_jobs += l.n;
      }
    HIPCHK(hipEventRecord(J.done, es));
    J.used = true;
    for (auto& up : live)
      if (up->grouped) HIPCHK(hipStreamWaitEvent(up->c->stream, J.done, 0));
  }
  // 3. the rest of the step, stage by stage over all runs
  for (auto& up : live) up->post_A();
  for (auto& up : live) up->stage1();
  for (auto& up : live) up->stage2();
  for (auto& up : live) up->stage3();
}

void pmchwt_server::engine_loop() {
  (void)hipSetDevice(device);
  std::vector<std::unique_ptr<ServeRun>> live;
  while (true) {
    {
      std::unique_lock<std::mutex> lk(m);
      cv_engine.wait(lk, [&] { return stop || !ready.empty() || !live.empty(); });
      if (stop) break;
      for (auto& r : ready) live.push_back(std::move(r));
      ready.clear();
      st.live = int64_t(live.size());
      st.max_live_seen = std::max<int64_t>(st.max_live_seen, int64_t(live.size()));
      st.rounds++;
    }
    // cancelled and finished runs leave before the round
    std::vector<std::unique_ptr<ServeRun>> keep;
    for (auto& up : live) {
      bool cancel;
      {
        std::lock_guard<std::mutex> lk(m);
        cancel = up->rec->cancel;
      }
      if (cancel || !up->stepping()) {
        std::lock_guard<std::mutex> lk(m);
        reap.push_back(std::move(up));
        cv_reap.notify_all();
      } else {
        keep.push_back(std::move(up));
      }
    }
    live.swap(keep);
    if (live.empty()) continue;
    try {
      round(live);
    } catch (const Fail& f) {
      // a device failure inside a round: fail every live request
      for (auto& up : live) {
        std::shared_ptr<ServeRecord> rec = up->rec;
        const int64_t est = rec->est;
        up.reset();
        {
          std::lock_guard<std::mutex> lk(m);
          live_count--;
          used -= est;
          err = f.msg;
        }
        complete(rec, f.code);
      }
      live.clear();
      cv_admit.notify_all();
    }
  }
  live.clear();  // shutting down: drop what is still live
}

extern "C" {

int pmchwt_server_create(pmchwt_server** out, int device, const pmchwt_server_opts* opts) {
  if (!out || !opts || opts->max_live < 1 || opts->max_live > 256 || opts->hbm_budget_bytes == 0)
    return PMCHWT_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PMCHWT_ERR_DEVICE;
  auto* s = new (std::nothrow) pmchwt_server();
  if (!s) return PMCHWT_ERR_OUT_OF_MEMORY;
  s->device = device;
  s->budget = opts->hbm_budget_bytes;
  s->max_live = opts->max_live;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s->es, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->jst[0].done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->jst[1].done, hipEventDisableTiming) != hipSuccess) {
    if (s->jst[0].done) (void)hipEventDestroy(s->jst[0].done);
    if (s->es) (void)hipStreamDestroy(s->es);
    delete s;
    return PMCHWT_ERR_DEVICE;
  }
  s->admit_thr = std::thread([s] { s->admit_loop(); });
  s->engine_thr = std::thread([s] { s->engine_loop(); });
  s->reap_thr = std::thread([s] { s->reap_loop(); });
  *out = s;
  return PMCHWT_OK;
}

int pmchwt_server_submit(pmchwt_server* s, const pmchwt_request* q, uint64_t* ticket) {
  if (!s || !q || !ticket || q->n_scatterers < 1 || !q->verts || !q->nv || !q->tris || !q->nt || !q->eps_r ||
      q->nrhs < 1 || !q->dirs || !q->pols || !(q->k_ext > 0) || q->precond < 0 || q->precond > 6)
    return PMCHWT_ERR_INVALID_ARG;
  const pmchwt_solver_opts& o = q->solver;
  if (!(o.tol > 0) || o.restart < 1 || o.restart > 1024 || o.max_iter < 1 || o.ir_max < 0)
    return PMCHWT_ERR_INVALID_ARG;
  auto rec = std::make_shared<ServeRecord>();
  for (int m = 0; m < q->n_scatterers; ++m) {
    if (!q->verts[m] || !q->tris[m] || q->nv[m] < 3 || q->nt[m] < 4) return PMCHWT_ERR_INVALID_MESH;
    rec->verts.emplace_back(q->verts[m], q->verts[m] + 3 * size_t(q->nv[m]));
    rec->tris.emplace_back(q->tris[m], q->tris[m] + 3 * size_t(q->nt[m]));
    rec->eps.push_back(q->eps_r[m]);
    for (int32_t v : rec->tris.back())
      if (v < 0 || v >= q->nv[m]) return PMCHWT_ERR_INVALID_MESH;
    if (q->nt[m] % 2 != 0) return PMCHWT_ERR_INVALID_MESH;  // closed triangulations have an even count
    rec->N += 3 * int64_t(q->nt[m]);
  }
  rec->k_ext = q->k_ext;
  rec->nrhs = q->nrhs;
  rec->dirs.assign(q->dirs, q->dirs + 3 * size_t(q->nrhs));
  rec->pols.assign(q->pols, q->pols + 3 * size_t(q->nrhs));
  rec->oA = q->opts_A;
  rec->oP = q->opts_P;
  rec->precond = q->precond;
  rec->so = q->solver;
  rec->est = serve_estimate(*rec);
  if (rec->est > int64_t(s->budget)) return PMCHWT_ERR_OVER_BUDGET;
  std::lock_guard<std::mutex> lk(s->m);
  rec->ticket = s->next_ticket++;
  rec->t_submit = now_ms();
  s->recs[rec->ticket] = rec;
  s->pending.push_back(rec);
  s->st.submitted++;
  *ticket = rec->ticket;
  s->cv_admit.notify_all();
  return PMCHWT_OK;
}

static void fill_result(const ServeRecord& r, pmchwt_result* res) {
  res->status = r.status;
  res->nrhs = r.nrhs;
  res->n_unknowns = r.N;
  res->device_bytes = r.est;
  res->ms_queued = r.t_admit > 0 ? r.t_admit - r.t_submit : now_ms() - r.t_submit;
  res->ms_total = r.t_done > 0 ? r.t_done - r.t_submit : 0.0;
  res->stats = r.stats;
}

int pmchwt_server_poll(pmchwt_server* s, uint64_t ticket, pmchwt_result* res) {
  if (!s || !res) return PMCHWT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return PMCHWT_ERR_INVALID_ARG;
  fill_result(*it->second, res);
  return PMCHWT_OK;
}

int pmchwt_server_wait(pmchwt_server* s, uint64_t ticket, double timeout_ms, pmchwt_result* res) {
  if (!s) return PMCHWT_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->m);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return PMCHWT_ERR_INVALID_ARG;
  std::shared_ptr<ServeRecord> rec = it->second;
  auto done = [&] { return rec->status != PMCHWT_PENDING && rec->status != PMCHWT_RUNNING; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, done);
  else
    s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done);
  if (res) fill_result(*rec, res);
  return done() ? PMCHWT_OK : PMCHWT_RUNNING;
}

int pmchwt_server_fetch(pmchwt_server* s, uint64_t ticket, pmchwt_complex* cur, double* sext, double* ssca) {
  if (!s) return PMCHWT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return PMCHWT_ERR_INVALID_ARG;
  ServeRecord& r = *it->second;
  if (r.status == PMCHWT_PENDING || r.status == PMCHWT_RUNNING) return PMCHWT_ERR_STATE;
  if (r.status == PMCHWT_OK || r.status == PMCHWT_ERR_NOT_CONVERGED) {
    if (cur) std::copy(r.currents.begin(), r.currents.end(), cur);
    if (sext) std::copy(r.sext.begin(), r.sext.end(), sext);
    if (ssca) std::copy(r.ssca.begin(), r.ssca.end(), ssca);
  }
  s->recs.erase(it);
  return PMCHWT_OK;
}

int pmchwt_server_cancel(pmchwt_server* s, uint64_t ticket) {
  if (!s) return PMCHWT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return PMCHWT_ERR_INVALID_ARG;
  it->second->cancel = true;
  s->cv_admit.notify_all();
  s->cv_engine.notify_all();
  return PMCHWT_OK;
}

int pmchwt_server_get_stats(pmchwt_server* s, pmchwt_server_stats* out) {
  if (!s || !out) return PMCHWT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->m);
  *out = s->st;
  out->pending = int64_t(s->pending.size());
  out->bytes_in_use = s->used;
  return PMCHWT_OK;
}

void pmchwt_server_destroy(pmchwt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
    for (auto& p : s->pending) p->status = PMCHWT_ERR_CANCELLED;
    s->pending.clear();
  }
  s->cv_admit.notify_all();
  s->cv_engine.notify_all();
  if (s->admit_thr.joinable()) s->admit_thr.join();
  if (s->engine_thr.joinable()) s->engine_thr.join();
  s->cv_reap.notify_all();
  if (s->reap_thr.joinable()) s->reap_thr.join();  // drains the runs handed over before the stop
  s->reap.clear();  // any run handed over after the reaper ended
  s->ready.clear();
  if (s->es) (void)hipStreamSynchronize(s->es);
  for (auto& J : s->jst) {
    J.h.reset();
    J.d = DBuf();
    if (J.done) (void)hipEventDestroy(J.done);
  }
  if (s->es) (void)hipStreamDestroy(s->es);
  delete s;
}

}  // extern "C"
