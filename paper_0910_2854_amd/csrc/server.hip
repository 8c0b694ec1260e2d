// server.hip -- request serving over a batch (include/fish.h, fish_server_*):
// a FIFO queue of simulation requests, admission while the batch's device
// pool has room, continuous batching (every resident box advances in the same
// launches; requests join and leave between chunks of steps), and retirement
// of finished boxes into the caller's output arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/fish.h"
#include "batch.h"
#include "engine.h"

using fish::Engine;

struct fish_server {
  fish_batch* batch = nullptr;
  int chunk = 8;
  int precision = 0, gravity = 0;
  size_t pool_bytes = 0;
  std::deque<fish_request> queue;
  struct Resident {
    fish_request req;
    int id;
    int left;
  };
  std::vector<Resident> resident;   // stepping
  std::vector<Resident> retiring;   // parked after their last chunk, read at the next call
  std::string err;
  long long steps_done = 0;      // double steps of all boxes, summed
  long long cell_steps = 0;      // cells x double steps, summed
};

namespace {

int sfail(fish_server* s, int code, const std::string& m) {
  s->err = m;
  return code;
}

}  // namespace

extern "C" {

int fish_server_create(const fish_batch_params* p, int chunk_steps, fish_server** out) {
  if (!out) return FISH_ERR_ARG;
  *out = nullptr;
  if (!p || chunk_steps < 1 || chunk_steps > 100000) return FISH_ERR_ARG;
  fish_server* s = new (std::nothrow) fish_server();
  if (!s) return FISH_ERR_NOMEM;
  int rc = fish_batch_create(p, &s->batch);
  if (rc) {
    delete s;
    return rc;
  }
  s->chunk = chunk_steps;
  s->precision = p->precision;
  s->gravity = p->gravity;
  s->pool_bytes = p->pool_bytes;
  *out = s;
  return FISH_OK;
}

void fish_server_destroy(fish_server* s) {
  if (!s) return;
  fish_batch_destroy(s->batch);
  delete s;
}

const char* fish_server_last_error(const fish_server* s) { return s ? s->err.c_str() : "null server"; }

fish_batch* fish_server_batch(fish_server* s) { return s ? s->batch : nullptr; }

int fish_server_submit(fish_server* s, const fish_request* r) {
  if (!s) return FISH_ERR_ARG;
  if (!r || !r->cell5 || !r->bx || !r->by || !r->bz || r->nsteps < 1) return sfail(s, FISH_ERR_ARG, "bad request");
  if (s->gravity && !r->phi) return sfail(s, FISH_ERR_ARG, "gravity needs phi");
  const int n[3] = {r->box.nx, r->box.ny, r->box.nz};
  const double h[3] = {r->box.dx, r->box.dy, r->box.dz};
  const int bc[3] = {r->box.bc[0], r->box.bc[1], r->box.bc[2]};
  if (Engine::validate_box(n, h, bc, r->box.cfl)) return sfail(s, FISH_ERR_ARG, "invalid box geometry");
  for (int a = 0; a < 3; ++a) {
    if (!r->widths[a]) continue;
    for (int i = 0; i < n[a]; ++i)
      if (!(r->widths[a][i] > 0.0) || !std::isfinite(r->widths[a][i]))
        return sfail(s, FISH_ERR_ARG, "widths must be finite and > 0");
  }
  if (fish_box_pool_bytes(&r->box, s->precision, s->gravity) > s->pool_bytes)
    return sfail(s, FISH_ERR_NOMEM, "request larger than the whole pool");
  s->queue.push_back(*r);
  return FISH_OK;
}

int fish_server_pump(fish_server* s, int64_t* done_tags, int32_t* done_status, int max_done, int* ndone) {
  if (!s || !ndone || (max_done > 0 && !done_tags)) return s ? sfail(s, FISH_ERR_ARG, "bad output") : FISH_ERR_ARG;
  *ndone = 0;
  Engine& e = s->batch->e;
  int rc;
  // 1. the next chunk of every stepping box (asynchronous); no box overshoots.
  //    Boxes done after it leave the launches at once (parked behind it) and
  //    are read at the next call, while the following chunk runs.
  std::vector<fish_server::Resident> finishing;
  if (!s->resident.empty()) {
    int k = s->chunk;
    for (const auto& x : s->resident) k = std::min(k, x.left);
    if ((rc = e.steps(k))) return sfail(s, rc, e.err);
    std::vector<fish_server::Resident> keep;
    for (auto& x : s->resident) {
      x.left -= k;
      s->cell_steps += (long long)k * x.req.box.nx * x.req.box.ny * x.req.box.nz;
      if (x.left > 0) {
        keep.push_back(x);
      } else {
        if ((rc = e.park(x.id))) return sfail(s, rc, e.err);
        finishing.push_back(x);
      }
    }
    s->resident.swap(keep);
    s->steps_done += k;
  }
  // 2. retire the boxes parked by the previous call: their reads wait for the
  //    chunk that finished them, not for the one just enqueued
  std::vector<fish_server::Resident> later;
  for (auto& x : s->retiring) {
    if (*ndone >= max_done) {
      later.push_back(x);  // report it at the next call
      continue;
    }
    fish::Scalars sc;
    if ((rc = e.read_scalars_parked(x.id, &sc))) return sfail(s, rc, e.err);
    if ((rc = e.download(x.id, x.req.out_cell5, x.req.out_bx, x.req.out_by, x.req.out_bz)))
      return sfail(s, rc, e.err);
    if ((rc = e.remove_box(x.id))) return sfail(s, rc, e.err);
    done_tags[*ndone] = x.req.tag;
    if (done_status) done_status[*ndone] = sc.status ? FISH_ERR_STATE : FISH_OK;
    ++*ndone;
  }
  s->retiring.swap(later);
  s->retiring.insert(s->retiring.end(), finishing.begin(), finishing.end());
  // 3. admission in arrival order while the head fits (no overtaking): host
  //    repacking and the copies overlap the chunk; the CFL check runs behind
  //    it.  A state that fails the check stops (dt = 0) and completes with
  //    FISH_ERR_STATE.
  bool added = false;
  while (!s->queue.empty()) {
    const fish_request& r = s->queue.front();
    const int n[3] = {r.box.nx, r.box.ny, r.box.nz};
    const double h[3] = {r.box.dx, r.box.dy, r.box.dz};
    const int bc[3] = {r.box.bc[0], r.box.bc[1], r.box.bc[2]};
    int id = -1;
    rc = e.add_box(n, h, bc, r.box.cfl, &id);
    if (rc == FISH_ERR_NOMEM) break;  // wait for a retirement
    if (rc) return sfail(s, rc, e.err);
    if ((rc = e.upload(id, r.cell5, r.bx, r.by, r.bz, r.phi))) return sfail(s, rc, e.err);
    for (int a = 0; a < 3; ++a)
      if (r.widths[a] && (rc = e.set_spacing(id, a, r.widths[a]))) return sfail(s, rc, e.err);
    s->resident.push_back({r, id, r.nsteps});
    s->queue.pop_front();
    added = true;
  }
  if (added && (rc = e.check_new())) return sfail(s, rc, e.err);
  return FISH_OK;
}

int fish_server_stats(const fish_server* s, int* queued, int* resident, size_t* pool_free, int64_t* cell_steps) {
  if (!s) return FISH_ERR_ARG;
  if (queued) *queued = (int)s->queue.size();
  if (resident) *resident = (int)s->resident.size();
  if (pool_free) *pool_free = fish_batch_free_bytes(s->batch);
  if (cell_steps) *cell_steps = s->cell_steps;
  return FISH_OK;
}

}  // extern "C"
