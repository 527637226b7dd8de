// server.cpp — continuous-batching step server over the cell API.
//
// Parameter queries (the many-query setting that motivates reduced models,
// Sec. 1 and Sec. 2.5) arrive as independent cells: a voxel image plus a
// parameter set plus a number of steps.  The server keeps every admitted
// cell's Newton state resident in device memory and advances all running
// cells together, one implicit Euler step per batched launch sequence
// (mbx_batch_step).  New requests join at the next step and finished ones
// leave after it (continuous batching).  Admission is first-come first-served
// against a device-memory budget: a request is admitted when its footprint
// fits next to the running cells.
//
// One worker thread owns the device work; submit / poll / result are
// thread-safe and never touch the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/mbx.h"

namespace mbx {
bool cutoff_reached(const mbx_params& p, double V);   // cell.cpp
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  std::vector<uint8_t> labels;
  int nx = 0, ny = 0, nz = 0;
  mbx_params p{};
  int n_steps = 0;
  int64_t footprint = 0;
  mbx_cell* cell = nullptr;
  mbx_request_info info{};
  std::vector<double> c, phi, n;   // final state (keep_state servers)
  std::string err;
};

// Interface-face counts from the labels (anode/pore and cathode/pore faces),
// for the footprint estimate at submission.
void count_faces(const uint8_t* lab, int nx, int ny, int nz, int64_t& fa, int64_t& fc) {
  fa = fc = 0;
  const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t i = x + sy * y + sz * z;
        const int L = lab[i];
        if (L == 0) continue;
        int nb = 0;
        if (x > 0 && lab[i - sx] == 0) ++nb;
        if (x + 1 < nx && lab[i + sx] == 0) ++nb;
        if (y > 0 && lab[i - sy] == 0) ++nb;
        if (y + 1 < ny && lab[i + sy] == 0) ++nb;
        if (z > 0 && lab[i - sz] == 0) ++nb;
        if (z + 1 < nz && lab[i + sz] == 0) ++nb;
        (L == 1 ? fa : fc) += nb;
      }
}

}  // namespace

struct mbx_server {
  int64_t budget = 0, used = 0;
  int precision = MBX_MIXED;
  double dt = 0.0;
  int keep_state = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;        // worker wake-up
  std::condition_variable idle_cv;   // drain waiters
  std::deque<Request*> queue;
  std::vector<Request*> running;     // touched by the worker only (read under mu by stats)
  int admitting = 0;                 // taken off the queue, cell not created yet (under mu)
  int retiring = 0;                  // left `running`, final state not yet copied out (under mu)
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_id = 1;
  bool stop = false;
  int64_t steps_run = 0, batches = 0;
  double busy_s = 0.0;
  std::thread worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void loop();
  void retire(Request* r, int status, bool was_running);
  bool idle() const { return queue.empty() && running.empty() && admitting == 0 && retiring == 0; }
};

// Copies a finished request's outputs, releases its cell and stamps its
// final status.  was_running: the request left `running` and is counted in
// `retiring` until this returns.
void mbx_server::retire(Request* r, int status, bool was_running) {
  if (r->cell) {
    double sac[2] = {0.0, 0.0};
    if (mbx_cell_mean_solid(r->cell, sac) == MBX_OK) {
      std::lock_guard<std::mutex> lk(mu);
      r->info.s_ac[0] = sac[0];
      r->info.s_ac[1] = sac[1];
    }
    if (keep_state && status == MBX_REQ_DONE) {
      int64_t N = 0, Fa = 0;
      mbx_cell_counts(r->cell, &N, &Fa, nullptr, nullptr);
      r->c.resize(N);
      r->phi.resize(N);
      r->n.resize(Fa);
      if (int e = mbx_cell_get_state(r->cell, r->c.data(), r->phi.data(), Fa ? r->n.data() : nullptr, 0)) {
        status = e;
        r->err = mbx_last_error();
      }
    }
    mbx_cell_destroy(r->cell);
    r->cell = nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  r->info.status = status;
  r->info.t_done = now();
  used -= r->footprint;
  if (was_running) --retiring;
}

void mbx_server::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (idle()) idle_cv.notify_all();
      cv.wait(lk, [&] { return stop || !queue.empty() || !running.empty(); });
      if (stop) break;
      // first-come first-served: the head waits until it fits
      while (!queue.empty() && used + queue.front()->footprint <= budget) {
        Request* r = queue.front();
        queue.pop_front();
        used += r->footprint;
        admit.push_back(r);
      }
      admitting += (int)admit.size();
    }
    for (Request* r : admit) {
      const int rc = mbx_cell_create(r->labels.data(), r->nx, r->ny, r->nz, &r->p, stream, &r->cell);
      if (rc != MBX_OK) {
        r->err = mbx_last_error();
        r->cell = nullptr;
        retire(r, rc, false);
        std::lock_guard<std::mutex> lk(mu);
        --admitting;
        continue;
      }
      std::vector<uint8_t>().swap(r->labels);   // the cell holds its own copy
      int64_t N = 0, Fa = 0;
      mbx_cell_counts(r->cell, &N, &Fa, nullptr, nullptr);
      std::lock_guard<std::mutex> lk(mu);
      r->info.status = MBX_REQ_RUNNING;
      r->info.t_admit = now();
      r->info.n_vox = N;
      r->info.n_an_faces = Fa;
      running.push_back(r);
      --admitting;
    }
    if (running.empty()) continue;
    const int n = (int)running.size();
    std::vector<mbx_cell*> cells(n);
    for (int i = 0; i < n; ++i) cells[i] = running[i]->cell;
    std::vector<int> st(n, 0);
    std::vector<mbx_step_info> inf(n);
    const double tb = now();
    int rc = mbx_batch_step(cells.data(), n, dt, st.data(), inf.data());
    const double te = now();
    std::string berr = rc != MBX_OK ? mbx_last_error() : "";
    std::vector<Request*> keep, done;
    {
      std::lock_guard<std::mutex> lk(mu);
      busy_s += te - tb;
      ++batches;
      for (int i = 0; i < n; ++i) {
        Request* r = running[i];
        const int s = rc != MBX_OK ? rc : st[i];
        bool cut = false;
        if (s == MBX_OK) {
          ++steps_run;
          r->info.steps_done++;
          r->info.V = inf[i].V;
          r->info.newton_iters += inf[i].newton_iters;
          r->info.krylov_iters += inf[i].krylov_iters;
          if (inf[i].substeps > 1) r->info.retried++;
          cut = mbx::cutoff_reached(r->p, inf[i].V);
          if (cut) r->info.cutoff = 1;
        } else {
          r->info.status = s;   // provisional; retire() stamps the time
          r->err = rc != MBX_OK ? berr : "step failed";
        }
        if (s != MBX_OK || cut || r->info.steps_done >= r->n_steps)
          done.push_back(r);
        else
          keep.push_back(r);
      }
      // requests leave `running` and enter `retiring` in one critical
      // section, so drain never sees the server idle in between
      running.swap(keep);
      retiring += (int)done.size();
    }
    for (Request* r : done) retire(r, r->info.status < 0 ? r->info.status : MBX_REQ_DONE, true);
  }
  // shutdown: release whatever is still resident
  for (Request* r : running)
    if (r->cell) mbx_cell_destroy(r->cell);
  running.clear();
}

extern "C" {

int mbx_server_create(int64_t budget_bytes, int precision, double dt, int keep_state, void* stream,
                      mbx_server** out) {
  if (!out) return MBX_EINVAL;
  *out = nullptr;
  if (budget_bytes <= 0 || !(dt > 0.0) || (precision != MBX_FP64 && precision != MBX_MIXED)) return MBX_EINVAL;
  auto* s = new mbx_server();
  s->budget = budget_bytes;
  s->precision = precision;
  s->dt = dt;
  s->keep_state = keep_state ? 1 : 0;
  s->stream = (hipStream_t)stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return MBX_EHIP;
  }
  s->t0 = Clock::now();
  s->worker = std::thread([s] { s->loop(); });
  *out = s;
  return MBX_OK;
}

int mbx_server_submit(mbx_server* s, const uint8_t* labels, int nx, int ny, int nz, const mbx_params* p,
                      int n_steps, int64_t* id) {
  if (!s || !labels || !p || !id || n_steps < 1 || nx < 1 || ny < 1 || nz < 2) return MBX_EINVAL;
  if (p->precision != s->precision) return MBX_EINVAL;
  const int64_t N = (int64_t)nx * ny * nz;
  if (N > (1 << 28)) return MBX_EINVAL;
  auto r = std::make_unique<Request>();
  r->labels.assign(labels, labels + N);
  r->nx = nx;
  r->ny = ny;
  r->nz = nz;
  r->p = *p;
  r->n_steps = n_steps;
  int64_t fa = 0, fc = 0;
  count_faces(labels, nx, ny, nz, fa, fc);
  r->footprint = mbx_cell_footprint(nx, ny, nz, p->precision, (int)fa, (int)fc);
  if (r->footprint < 0) return MBX_EINVAL;
  if (r->footprint > s->budget) return MBX_EBUDGET;
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->info.status = MBX_REQ_QUEUED;
  r->info.t_submit = s->now();
  *id = r->id;
  s->queue.push_back(r.get());
  s->all.emplace(r->id, std::move(r));
  s->cv.notify_one();
  return MBX_OK;
}

int mbx_server_error(mbx_server* s, int64_t id, char* buf, int len) {
  if (!s || !buf || len < 1) return MBX_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return MBX_EINVAL;
  const Request& r = *it->second;
  const std::string& e = r.info.status < 0 ? r.err : std::string();
  const size_t n = std::min(e.size(), (size_t)len - 1);
  memcpy(buf, e.data(), n);
  buf[n] = '\0';
  return MBX_OK;
}

int mbx_server_poll(mbx_server* s, int64_t id, mbx_request_info* info) {
  if (!s || !info) return MBX_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return MBX_EINVAL;
  *info = it->second->info;
  return MBX_OK;
}

int mbx_server_result(mbx_server* s, int64_t id, double* cfield, double* phi, double* n_pl) {
  if (!s) return MBX_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return MBX_EINVAL;
  const Request& r = *it->second;
  if (!s->keep_state || r.info.status != MBX_REQ_DONE) return MBX_ESTATE;
  if (cfield) std::memcpy(cfield, r.c.data(), 8 * r.c.size());
  if (phi) std::memcpy(phi, r.phi.data(), 8 * r.phi.size());
  if (n_pl && !r.n.empty()) std::memcpy(n_pl, r.n.data(), 8 * r.n.size());
  return MBX_OK;
}

int mbx_server_drain(mbx_server* s, double timeout_s) {
  if (!s) return MBX_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return s->idle(); });
  return ok ? MBX_OK : MBX_ESTATE;
}

double mbx_server_clock(const mbx_server* s) { return s ? s->now() : 0.0; }

int mbx_server_stats(mbx_server* s, mbx_server_info* out) {
  if (!s || !out) return MBX_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->steps_run = s->steps_run;
  out->batches = s->batches;
  out->busy_s = s->busy_s;
  out->bytes_in_use = s->used;
  out->running = (int)s->running.size();
  out->queued = (int)s->queue.size();
  return MBX_OK;
}

void mbx_server_destroy(mbx_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  delete s;
}

}  // extern "C"
