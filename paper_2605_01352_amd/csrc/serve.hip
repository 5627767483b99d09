// Serving loop with continuous batching: rollout requests queue up, are
// admitted into free env slots of one resident world as capacity and the HBM
// budget allow, step together in the co-scheduled loop, and leave when their
// horizon is reached, freeing their slots for the next ones.
//
// The loop is pipelined.  A tick enqueues k iterations of the schedule over
// every running request (k = the fewest steps any of them has left, at most
// kTickIters) and records events; it does not wait for them.  Up to
// kInflight ticks run ahead of the host, which meanwhile admits new requests
// (their uploads go to free memory, beside the running kernels) and retires
// finished ones: a request whose last step is enqueued leaves every later
// launch at once, and its memory is released when the events of its last
// tick have completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "vuda.h"
#include "vuda_runtime.h"

using namespace vuda;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Owned copy of a request's env batch.
struct Batch {
  int32_t n_envs = 0;
  std::vector<int32_t> body_off, cam_off, cam_w, cam_h;
  std::vector<uint8_t> type, albedo;
  std::vector<float> size, rbound, inv_m, inv_I, pos, vel, quat, omega, cam_vp;
  std::vector<float> ext, inertia;  // empty when the batch has no box

  void copy_from(const vuda_env_batch& b) {
    n_envs = b.n_envs;
    const int64_t nb = b.body_off[b.n_envs];
    const int32_t nc = b.cam_off[b.n_envs];
    body_off.assign(b.body_off, b.body_off + b.n_envs + 1);
    cam_off.assign(b.cam_off, b.cam_off + b.n_envs + 1);
    type.assign(b.type, b.type + nb);
    albedo.assign(b.albedo, b.albedo + nb);
    size.assign(b.size, b.size + nb);
    rbound.assign(b.rbound, b.rbound + nb);
    inv_m.assign(b.inv_m, b.inv_m + nb);
    inv_I.assign(b.inv_I, b.inv_I + nb);
    pos.assign(b.pos, b.pos + 3 * nb);
    vel.assign(b.vel, b.vel + 3 * nb);
    quat.assign(b.quat, b.quat + 4 * nb);
    omega.assign(b.omega, b.omega + 3 * nb);
    cam_vp.assign(b.cam_vp, b.cam_vp + 16 * (size_t)nc);
    cam_w.assign(b.cam_w, b.cam_w + nc);
    cam_h.assign(b.cam_h, b.cam_h + nc);
    ext.clear();
    inertia.clear();
    if (b.ext && b.inertia) {
      ext.assign(b.ext, b.ext + 3 * nb);
      inertia.assign(b.inertia, b.inertia + 3 * nb);
    }
  }
  vuda_env_batch view() const {
    vuda_env_batch b{};
    b.n_envs = n_envs;
    b.body_off = body_off.data();
    b.type = type.data(); b.size = size.data(); b.rbound = rbound.data();
    b.inv_m = inv_m.data(); b.inv_I = inv_I.data(); b.albedo = albedo.data();
    b.pos = pos.data(); b.vel = vel.data(); b.quat = quat.data(); b.omega = omega.data();
    b.cam_off = cam_off.data(); b.cam_vp = cam_vp.data(); b.cam_w = cam_w.data(); b.cam_h = cam_h.data();
    b.ext = ext.empty() ? nullptr : ext.data();
    b.inertia = inertia.empty() ? nullptr : inertia.data();
    return b;
  }
  int64_t bodies() const { return body_off.empty() ? 0 : body_off.back(); }
  int64_t pixels() const {
    int64_t p = 0;
    for (size_t c = 0; c < cam_w.size(); ++c) p += (int64_t)cam_w[c] * cam_h[c];
    return p;
  }
};

struct Request {
  int64_t id = 0;
  Batch batch;
  int32_t horizon = 0;
  int32_t steps = 0;     // steps enqueued
  int32_t first_env = -1;
  bool retired = false;  // every step enqueued; waiting for its last tick
  double t_submit = 0.0, t_admit = 0.0;
  uint64_t bytes = 0;
};

// Ticks enqueued ahead of the host, and iterations per tick.
constexpr int kInflight = 2;
constexpr int32_t kTickIters = 8;

// One enqueued tick: events that complete with its work, the requests whose
// last step it holds, and the env-steps it serves.
struct Tick {
  hipEvent_t ev[2] = {nullptr, nullptr};
  int nev = 0;
  std::vector<int32_t> finishing;  // first env slot of each
  int64_t env_steps = 0;
};

struct Result {
  std::vector<float> state;
  std::vector<uint8_t> rgb;
  std::vector<uint32_t> depth;
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct vuda_server {
  vuda_world* w = nullptr;
  int32_t sched = VUDA_SCHED_INTERSTEP;
  bool keep = false;
  int parity = 0;  // step parity shared by every active env at a tick boundary
  uint64_t budget = 0, reserved = 0, peak_reserved = 0;
  std::deque<Request> queue;
  std::map<int32_t, Request> active;  // by first env slot
  std::deque<std::pair<int64_t, double>> done;
  std::map<int64_t, Result> results;
  std::vector<double> latencies, queue_delays;
  int64_t submitted = 0, admitted = 0, completed = 0, env_steps = 0, ticks = 0, rejected = 0;
  double busy = 0.0;
  std::deque<Tick> inflight;
  std::vector<hipEvent_t> spare;  // events of reaped ticks, for reuse

  // Completes the oldest enqueued tick (waiting for it if `block`): its
  // env-steps count as served and its finishing requests are released.
  // Returns 1 if a tick was reaped, 0 if it is still running, < 0 on error.
  int reap(bool block, int32_t* ncomp);

  // Device bytes a request holds while resident: both state buffers and the
  // static arrays per body, the primitive/vertex maps, the RGB-D images and
  // the raster scratch of its cameras.
  uint64_t request_bytes(const Batch& b) const {
    const int64_t nb = b.bodies();
    int64_t maps = 0;
    for (int32_t e = 0; e < b.n_envs; ++e) {
      maps += 2 * 16 + w->tpl.ground_nf + w->tpl.ground_nv;
      for (int32_t i = b.body_off[e]; i < b.body_off[e + 1]; ++i)
        maps += b.type[i] ? w->tpl.cube_nf + w->tpl.cube_nv : w->tpl.sphere_nf + w->tpl.sphere_nv;
    }
    return (uint64_t)nb * (2 * 4 * kStateComps + 50) + (uint64_t)maps + (uint64_t)b.pixels() * 7 +
           (uint64_t)b.n_envs * sizeof(EnvDev) + b.cam_w.size() * sizeof(CamDev) +
           256 * (uint64_t)w->rs_units(b.view());
  }
};

extern "C" int vuda_serve_create(const vuda_world_desc* desc, float cu_split, int32_t schedule,
                                 int32_t keep_results, vuda_server** out) {
  if (!desc || !out) return fail(VUDA_EINVAL, "null argument");
  if (schedule < VUDA_SCHED_SERIAL || schedule > VUDA_SCHED_PIPELINED)
    return fail(VUDA_EINVAL, "schedule %d", schedule);
  *out = nullptr;
  vuda_server* s = new (std::nothrow) vuda_server();
  if (!s) return fail(VUDA_ENOMEM, "host allocation");
  vuda_world_desc d = *desc;
  d.hbm_budget = 0;  // the budget bounds the admitted requests, not the arena
  int rc = vuda_create_world(&d, nullptr, &s->w);
  if (!rc) rc = vuda_cosched(s->w, cu_split);
  if (rc) {
    if (s->w) vuda_destroy_world(s->w);
    delete s;
    return rc;
  }
  s->sched = schedule;
  s->keep = keep_results != 0;
  s->budget = desc->hbm_budget;
  *out = s;
  return VUDA_OK;
}

extern "C" int vuda_serve_destroy(vuda_server* s) {
  if (!s) return fail(VUDA_EINVAL, "null server");
  while (s->reap(true, nullptr) == 1) {
  }
  for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
  for (Tick& t : s->inflight)
    for (hipEvent_t e : t.ev)
      if (e) (void)hipEventDestroy(e);
  int rc = vuda_destroy_world(s->w);
  delete s;
  return rc;
}

extern "C" int vuda_serve_world(vuda_server* s, vuda_world** w) {
  if (!s || !w) return fail(VUDA_EINVAL, "null argument");
  *w = s->w;
  return VUDA_OK;
}

extern "C" int vuda_serve_submit(vuda_server* s, int64_t id, const vuda_env_batch* b, int32_t horizon) {
  if (!s || !b) return fail(VUDA_EINVAL, "null argument");
  if (horizon < 1) return fail(VUDA_EINVAL, "horizon %d", horizon);
  if (b->n_envs < 1 || !b->body_off || !b->cam_off) return fail(VUDA_EINVAL, "empty request");
  // a request is checked here, so that the queue never holds one that
  // admission would refuse for good
  vuda_render_desc rd{};
  rd.ground_nf = s->w->tpl.ground_nf;
  rd.sphere_nf = s->w->tpl.sphere_nf;
  rd.cube_nf = s->w->tpl.cube_nf;
  int64_t nb = 0, npix = 0;
  int32_t nc = 0;
  int rc = validate_batch(*b, rd, &nb, &nc, &npix);
  if (rc) return rc;
  int64_t nprim = 0, nvert = 0;
  s->w->map_sizes(*b, &nprim, &nvert);
  if (b->n_envs > s->w->cap_envs || nb > s->w->cap_bodies || nc > s->w->cap_cams || npix > s->w->cap_pixels ||
      nprim > s->w->cap_prims || nvert > s->w->cap_verts || s->w->rs_units(*b) > s->w->cap_rs)
    return fail(VUDA_EINVAL, "request of %d envs, %lld bodies, %d cameras, %lld pixels exceeds the world's capacity",
                b->n_envs, (long long)nb, nc, (long long)npix);
  Request r;
  r.id = id;
  r.horizon = horizon;
  r.batch.copy_from(*b);
  r.bytes = s->request_bytes(r.batch);
  if (s->budget && r.bytes > s->budget)
    return fail(VUDA_EINVAL, "request of %llu bytes can never fit the budget", (unsigned long long)r.bytes);
  r.t_submit = now_s();
  s->queue.push_back(std::move(r));
  ++s->submitted;
  return VUDA_OK;
}

int vuda_server::reap(bool block, int32_t* ncomp) {
  if (inflight.empty()) return 0;
  Tick& t = inflight.front();
  for (int k = 0; k < t.nev; ++k) {
    const hipError_t q = block ? hipEventSynchronize(t.ev[k]) : hipEventQuery(t.ev[k]);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return hip_fail(q, "tick event");
  }
  int rc = w->check_flags();
  if (rc) return rc;
  env_steps += t.env_steps;
  ++ticks;
  const double now = now_s();
  for (int32_t first : t.finishing) {
    Request& r = active[first];
    rc = vuda_release(w, r.first_env, r.batch.n_envs);
    if (rc) return rc;
    const double lat = now - r.t_submit;
    latencies.push_back(lat);
    done.push_back({r.id, lat});
    reserved -= r.bytes;
    ++completed;
    if (ncomp) ++*ncomp;
    active.erase(first);
  }
  for (int k = 0; k < 2; ++k)
    if (t.ev[k]) spare.push_back(t.ev[k]);
  inflight.pop_front();
  return 1;
}

extern "C" int vuda_serve_tick(vuda_server* s, int32_t* n_completed) {
  if (!s) return fail(VUDA_EINVAL, "null server");
  const double t0 = now_s();
  int32_t ncomp = 0;
  // 1. ticks that have finished, then room for one more in flight
  int rc;
  while ((rc = s->reap(false, &ncomp)) == 1) {
  }
  if (rc < 0) return rc;
  while ((int)s->inflight.size() >= kInflight) {
    rc = s->reap(true, &ncomp);
    if (rc < 0) return rc;
  }
  // 2. admission in FIFO order while the budget and the world's capacity
  // allow; the new envs start from the step parity every running env has
  // after the enqueued ticks
  while (!s->queue.empty()) {
    Request& r = s->queue.front();
    if (s->budget && s->reserved + r.bytes > s->budget) break;
    const vuda_env_batch view = r.batch.view();
    int32_t first = -1;
    rc = vuda_admit(s->w, &view, s->parity, &first);
    if (rc == VUDA_EBUSY) break;
    if (rc) {
      // refused for good (submit checks make this rare): drop it, go on
      ++s->rejected;
      s->queue.pop_front();
      continue;
    }
    r.first_env = first;
    r.t_admit = now_s();
    s->queue_delays.push_back(r.t_admit - r.t_submit);
    s->reserved += r.bytes;
    s->peak_reserved = std::max(s->peak_reserved, s->reserved);
    ++s->admitted;
    Request moved = std::move(r);
    s->queue.pop_front();
    s->active.emplace(moved.first_env, std::move(moved));
  }
  // 3. k co-scheduled iterations over every running request, k the fewest
  // steps one of them has left (at most kTickIters)
  int32_t k = kTickIters;
  int64_t envs = 0;
  for (auto& kv : s->active)
    if (!kv.second.retired) {
      k = std::min(k, kv.second.horizon - kv.second.steps);
      envs += kv.second.batch.n_envs;
    }
  if (envs > 0) {
    rc = vuda_run(s->w, s->sched, k);
    if (rc) return rc;
    s->parity ^= (k & 1);
    Tick t;
    t.env_steps = envs * k;
    for (auto& kv : s->active) {
      Request& r = kv.second;
      if (r.retired) continue;
      r.steps += k;
      if (r.steps < r.horizon) continue;
      const int32_t lo = r.first_env, hi = r.first_env + r.batch.n_envs;
      if (s->keep) {
        // the final state and a frame of it
        Result res;
        size_t nbytes = 0;
        rc = vuda_render(s->w, lo, hi);
        if (!rc) rc = vuda_fetch_bytes(s->w, VUDA_FETCH_STATE, lo, hi, &nbytes);
        if (!rc) {
          res.state.resize(nbytes / 4);
          rc = vuda_fetch(s->w, VUDA_FETCH_STATE, lo, hi, res.state.data(), nbytes, 0);
        }
        if (!rc) rc = vuda_fetch_bytes(s->w, VUDA_FETCH_RGB, lo, hi, &nbytes);
        if (!rc) {
          res.rgb.resize(nbytes);
          rc = vuda_fetch(s->w, VUDA_FETCH_RGB, lo, hi, res.rgb.data(), nbytes, 0);
        }
        if (!rc) rc = vuda_fetch_bytes(s->w, VUDA_FETCH_DEPTH, lo, hi, &nbytes);
        if (!rc) {
          res.depth.resize(nbytes / 4);
          rc = vuda_fetch(s->w, VUDA_FETCH_DEPTH, lo, hi, res.depth.data(), nbytes, 0);
        }
        if (rc) return rc;
        s->results[r.id] = std::move(res);
      }
      // no later launch includes its envs; the memory is released once
      // this tick has run
      rc = s->w->retire(lo, r.batch.n_envs);
      if (rc) return rc;
      r.retired = true;
      t.finishing.push_back(kv.first);
    }
    for (int q = 0; q < 2; ++q) {
      if (!s->spare.empty()) {
        t.ev[q] = s->spare.back();
        s->spare.pop_back();
      }
    }
    t.nev = s->w->mark(t.ev);
    if (t.nev < 0) return VUDA_EHIP;
    s->inflight.push_back(std::move(t));
  } else {
    // nothing running: finish what is in flight
    while ((rc = s->reap(true, &ncomp)) == 1) {
    }
    if (rc < 0) return rc;
  }
  s->busy += now_s() - t0;
  if (n_completed) *n_completed = ncomp;
  return VUDA_OK;
}

extern "C" int vuda_serve_completed(vuda_server* s, int64_t* ids, double* lat, int32_t cap, int32_t* n) {
  if (!s || !n || (cap > 0 && (!ids || !lat))) return fail(VUDA_EINVAL, "null argument");
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    ids[k] = s->done.front().first;
    lat[k] = s->done.front().second;
    s->done.pop_front();
    ++k;
  }
  *n = k;
  return VUDA_OK;
}

extern "C" int vuda_serve_result(vuda_server* s, int64_t id, int32_t what, void* dst, size_t bytes,
                                 size_t* need) {
  if (!s) return fail(VUDA_EINVAL, "null server");
  auto it = s->results.find(id);
  if (it == s->results.end()) return fail(VUDA_EINVAL, "no kept result for request %lld", (long long)id);
  const void* src = nullptr;
  size_t n = 0;
  switch (what) {
    case VUDA_FETCH_STATE: src = it->second.state.data(); n = 4 * it->second.state.size(); break;
    case VUDA_FETCH_RGB: src = it->second.rgb.data(); n = it->second.rgb.size(); break;
    case VUDA_FETCH_DEPTH: src = it->second.depth.data(); n = 4 * it->second.depth.size(); break;
    default: return fail(VUDA_EINVAL, "result selector %d", what);
  }
  if (need) *need = n;
  if (!dst) return VUDA_OK;
  if (bytes < n) return fail(VUDA_EINVAL, "dst holds %zu bytes, need %zu", bytes, n);
  memcpy(dst, src, n);
  return VUDA_OK;
}

extern "C" int vuda_serve_stats(vuda_server* s, vuda_serve_stats_t* o) {
  if (!s || !o) return fail(VUDA_EINVAL, "null argument");
  memset(o, 0, sizeof(*o));
  o->submitted = s->submitted;
  o->admitted = s->admitted;
  o->completed = s->completed;
  o->queued = (int64_t)s->queue.size();
  o->active_requests = (int64_t)s->active.size();
  for (auto& kv : s->active) o->active_envs += kv.second.batch.n_envs;
  o->env_steps = s->env_steps;
  o->ticks = s->ticks;
  o->busy_s = s->busy;
  o->latency_p50_s = percentile(s->latencies, 0.50);
  o->latency_p99_s = percentile(s->latencies, 0.99);
  o->latency_max_s = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
  double m = 0.0;
  for (double x : s->latencies) m += x;
  o->latency_mean_s = s->latencies.empty() ? 0.0 : m / (double)s->latencies.size();
  o->queue_p50_s = percentile(s->queue_delays, 0.50);
  o->queue_p99_s = percentile(s->queue_delays, 0.99);
  o->reserved_bytes = s->reserved;
  o->peak_reserved_bytes = s->peak_reserved;
  o->rejected = s->rejected;
  return VUDA_OK;
}
