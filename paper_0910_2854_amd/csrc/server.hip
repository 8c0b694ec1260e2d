// server.hip -- request serving over a batch (include/fish.h, fish_server_*):
// a FIFO queue of simulation requests, admission while the batch's device
// pool has room, continuous batching (every resident box advances in the same
// launches; requests join and leave between chunks of steps), and retirement
// of finished boxes into the caller's output arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/fish.h"
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
  std::vector<Resident> resident;
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
  if (fish_box_pool_bytes(&r->box, s->precision, s->gravity) > s->pool_bytes)
    return sfail(s, FISH_ERR_NOMEM, "request larger than the whole pool");
  s->queue.push_back(*r);
  return FISH_OK;
}

int fish_server_pump(fish_server* s, int64_t* done_tags, int32_t* done_status, int max_done, int* ndone) {
  if (!s || !ndone || (max_done > 0 && !done_tags)) return s ? sfail(s, FISH_ERR_ARG, "bad output") : FISH_ERR_ARG;
  *ndone = 0;
  // 1. the next chunk of steps of every resident box, enqueued first so that
  //    the host work of the admissions below overlaps it; no box overshoots
  int k = 0;
  if (!s->resident.empty()) {
    k = s->chunk;
    for (const auto& x : s->resident) k = std::min(k, x.left);
    int rc = fish_batch_step(s->batch, k);
    if (rc) return sfail(s, rc, fish_batch_last_error(s->batch));
  }
  const size_t stepped = s->resident.size();
  // 2. admission in arrival order while the head fits (no overtaking); the
  //    new boxes take no step of this chunk
  while (!s->queue.empty()) {
    const fish_request& r = s->queue.front();
    int id = -1;
    int rc = fish_batch_add(s->batch, &r.box, r.cell5, r.bx, r.by, r.bz, r.phi, &id);
    if (rc == FISH_ERR_NOMEM) break;  // wait for a retirement
    if (rc != FISH_OK) {
      // a request whose state fails the check completes at once with its status
      if (*ndone >= max_done) return sfail(s, FISH_ERR_ARG, "done buffer too small");
      done_tags[*ndone] = r.tag;
      if (done_status) done_status[*ndone] = rc;
      ++*ndone;
      s->queue.pop_front();
      continue;
    }
    s->resident.push_back({r, id, r.nsteps});
    s->queue.pop_front();
  }
  for (size_t i = 0; i < stepped; ++i) {
    auto& x = s->resident[i];
    x.left -= k;
    s->cell_steps += (long long)k * x.req.box.nx * x.req.box.ny * x.req.box.nz;
  }
  s->steps_done += k;
  // 3. retire finished boxes (their downloads wait for the chunk)
  std::vector<fish_server::Resident> keep;
  keep.reserve(s->resident.size());
  for (auto& x : s->resident) {
    if (x.left > 0) {
      keep.push_back(x);
      continue;
    }
    if (*ndone >= max_done) {
      keep.push_back(x);  // report it at the next pump
      continue;
    }
    double t = 0.0;
    int st = fish_batch_get(s->batch, x.id, x.req.out_cell5, x.req.out_bx, x.req.out_by, x.req.out_bz, &t);
    if (st != FISH_OK && st != FISH_ERR_STATE) return sfail(s, st, fish_batch_last_error(s->batch));
    int rc = fish_batch_remove(s->batch, x.id);
    if (rc) return sfail(s, rc, fish_batch_last_error(s->batch));
    done_tags[*ndone] = x.req.tag;
    if (done_status) done_status[*ndone] = st;
    ++*ndone;
  }
  s->resident.swap(keep);
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
