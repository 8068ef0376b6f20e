// Tracking service with continuous batching, behind the C ABI of acopf.h.
//
// The paper motivates fast tracking of the ACOPF optimum as loads change
// (Sec. I, Sec. IV-C): each new load picture is solved warm from the previous
// solution. A server keeps several grids resident on one GPU and solves a
// stream of such requests. It is written against the library's own entry
// points (one handle, per-grid start/run/poll, device-side copies); every
// step of a solve runs in the kernels behind them.
//
// Layout: the handle holds, for every resident grid j, 1 + k_j instances of
// the same grid data. One of them is the grid's home (its last committed ADMM
// state); the others are free slots. The k_j are chosen so that the device
// footprint of all instances fits the HBM budget: round robin over the grids,
// smallest first, one slot at a time, while the budget allows.
//
// A request (grid j, new loads) is admitted between iteration chunks as soon
// as a slot of grid j is free: the home state is copied into the slot on the
// device, the loads are set, and a warm start joins the running launches, so
// its inner iterations overlap with those of every other request in flight.
// When it finishes, its slot becomes the grid's home and the previous home a
// free slot, so a completion copies nothing. A grid whose budget allows no
// slot runs its requests on its home instance, one at a time.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/acopf.h"

namespace acopf_dev {
int report_error(int code, const char* msg);  // sets acopf_last_error's text
}

namespace {

int fail(int code, const char* msg) { return acopf_dev::report_error(code, msg); }

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Device footprint of one grid instance in the library's layout: the coupling
// vectors, the branch data, state and records, the second buffer of the
// branch step's results, the generator and bus arrays, their indices and the
// residual history.
double instance_bytes(const acopf_grid& g) {
  const double nb = g.n_bus, ng = g.n_gen, nl = g.n_branch;
  const double m = 2 * ng + 8 * nl;
  const double doubles =
      5 * m + 9 * nl + 8 * nl + 5 * nl + 16 * nl + (m + 10 * nl) + 9 * ng + 6 * nb;
  const double ints = 2 * nl + nl + 2 * nl + 2 * nl + ng + 3 * nb + 4;
  return 8 * doubles + 4 * ints + 6.0 * 8 * (1 << 15);
}

struct Pending {
  int64_t id;
  std::vector<double> pd, qd;
  double submitted;
};

struct Running {
  int64_t id;
  int grid;
  double submitted, admitted;
};

}  // namespace

struct acopf_server_s {
  acopf_handle h = nullptr;
  int G = 0;
  int chunk = 16;
  std::vector<int> nbus;
  std::vector<int> slots;              // slot instances of each grid
  std::vector<int> home;               // instance holding each grid's committed state
  std::vector<std::deque<int>> free;   // free slot instances of each grid
  std::vector<char> home_busy;         // a grid without slots is running on its home
  std::vector<std::deque<Pending>> queue;
  std::map<int, Running> inflight;     // instance -> request
  std::deque<acopf_served> done;
  std::vector<acopf_result> cold;      // the cold solve of each home
  double bytes_used = 0.0;
  int64_t queued = 0;
};

extern "C" {

int acopf_serving_plan(const acopf_grid* grids, int32_t n_grids, double budget_bytes,
                       int32_t max_slots, int32_t* slots_out, double* bytes_used) {
  if (!grids || n_grids < 1 || !slots_out || max_slots < 0)
    return fail(ACOPF_EINVAL, "serving_plan: need grids, n_grids >= 1, an output, max_slots >= 0");
  std::vector<double> size(n_grids);
  double homes = 0.0;
  for (int j = 0; j < n_grids; ++j) {
    size[j] = instance_bytes(grids[j]);
    homes += size[j];
    slots_out[j] = 0;
  }
  if (!(budget_bytes >= homes))
    return fail(ACOPF_EBUDGET, ("HBM budget of " + std::to_string(budget_bytes) +
                                " bytes below the resident grids' " + std::to_string(homes))
                                   .c_str());
  std::vector<int> order(n_grids);
  for (int j = 0; j < n_grids; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size[a] < size[b]; });
  double used = homes;
  for (bool grew = true; grew;) {
    grew = false;
    for (int j : order)
      if (slots_out[j] < max_slots && used + size[j] <= budget_bytes) {
        ++slots_out[j];
        used += size[j];
        grew = true;
      }
  }
  if (bytes_used) *bytes_used = used;
  return ACOPF_OK;
}

int acopf_server_create(const acopf_grid* grids, int32_t n_grids, const acopf_params* params,
                        double budget_bytes, int32_t max_slots, int32_t chunk, int32_t device,
                        acopf_server* out) {
  if (!grids || n_grids < 1 || !out || max_slots < 0 || chunk < 0)
    return fail(ACOPF_EINVAL, "server_create: need grids, n_grids >= 1, an output, max_slots >= 0, chunk >= 0");
  *out = nullptr;
  if (!(budget_bytes > 0.0)) {
    int64_t mem[2] = {0, 0};
    int rc = acopf_device_memory(device, mem);
    if (rc) return rc;
    budget_bytes = 0.9 * (double)mem[0];
  }
  acopf_server s = new acopf_server_s();
  s->G = n_grids;
  s->slots.resize(n_grids);
  int rc = acopf_serving_plan(grids, n_grids, budget_bytes, max_slots, s->slots.data(),
                              &s->bytes_used);
  if (rc) {
    delete s;
    return rc;
  }
  // instances: the homes 0..G-1, then each grid's slots
  std::vector<acopf_grid> inst(grids, grids + n_grids);
  s->free.resize(n_grids);
  for (int j = 0; j < n_grids; ++j)
    for (int k = 0; k < s->slots[j]; ++k) {
      s->free[j].push_back((int)inst.size());
      inst.push_back(grids[j]);
    }
  rc = acopf_create(inst.data(), (int32_t)inst.size(), params, device, nullptr, &s->h);
  if (rc) {
    delete s;
    return rc;
  }
  // one launch lane: at the served rates a few requests are in flight, and
  // launching them as one group admits and retires them at the lowest
  // latency (measured: p50 2.89 against 3.0 ms at 200 requests/s with two)
  acopf_tuning t;
  rc = acopf_get_tuning(s->h, &t);
  if (!rc && ((chunk > 0 && chunk != t.chunk) || t.lanes != 1)) {
    if (chunk > 0) t.chunk = chunk;
    t.lanes = 1;
    rc = acopf_set_tuning(s->h, &t);
  }
  s->chunk = chunk > 0 ? chunk : t.chunk;
  for (int j = 0; !rc && j < n_grids; ++j) {
    s->nbus.push_back(grids[j].n_bus);
    s->home.push_back(j);
    rc = acopf_start(s->h, j, ACOPF_COLD, 0);
  }
  for (int32_t running = 1; !rc && running > 0;) rc = acopf_run(s->h, 1 << 16, &running);
  s->cold.resize(n_grids);
  for (int j = 0; !rc && j < n_grids; ++j) rc = acopf_poll(s->h, j, nullptr, &s->cold[j]);
  if (rc) {
    acopf_destroy(s->h);
    delete s;
    return rc;
  }
  s->home_busy.assign(n_grids, 0);
  s->queue.resize(n_grids);
  *out = s;
  return ACOPF_OK;
}

int acopf_server_submit(acopf_server s, int32_t grid, const double* pd, const double* qd,
                        int64_t request_id) {
  if (!s || grid < 0 || grid >= s->G || !pd || !qd)
    return fail(ACOPF_EINVAL, "server_submit: null server or loads, or grid out of range");
  const int n = s->nbus[grid];
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(pd[i]) || !std::isfinite(qd[i]))
      return fail(ACOPF_EINVAL, "server_submit: non-finite load");
  s->queue[grid].push_back(Pending{request_id, std::vector<double>(pd, pd + n),
                                   std::vector<double>(qd, qd + n), now_seconds()});
  ++s->queued;
  return ACOPF_OK;
}

int acopf_server_step(acopf_server s, int32_t* in_flight, int32_t* queued) {
  if (!s) return fail(ACOPF_EINVAL, "null server");
  int rc = ACOPF_OK;
  // admission: every grid's queue, in arrival order, while instances are free
  for (int j = 0; j < s->G && !rc; ++j) {
    while (!s->queue[j].empty()) {
      int k;
      if (s->slots[j] > 0) {
        if (s->free[j].empty()) break;
        k = s->free[j].front();
        rc = acopf_copy_grid(s->h, s->home[j], k);
        if (rc) break;
        s->free[j].pop_front();
      } else {
        if (s->home_busy[j]) break;
        k = s->home[j];
        s->home_busy[j] = 1;
      }
      Pending& p = s->queue[j].front();
      rc = acopf_update_loads(s->h, k, p.pd.data(), p.qd.data());
      if (!rc) rc = acopf_start(s->h, k, ACOPF_WARM, 0);
      if (rc) break;
      s->inflight[k] = Running{p.id, j, p.submitted, now_seconds()};
      s->queue[j].pop_front();
      --s->queued;
    }
  }
  if (!rc && !s->inflight.empty()) {
    int32_t running = 0;
    rc = acopf_run(s->h, s->chunk, &running);
    // retire the requests whose instance finished; the instance becomes home
    for (auto it = s->inflight.begin(); !rc && it != s->inflight.end();) {
      int32_t is_running = 0;
      rc = acopf_poll(s->h, it->first, &is_running, nullptr);
      if (rc || is_running) {
        ++it;
        continue;
      }
      acopf_served d{};
      d.request_id = it->second.id;
      d.grid = it->second.grid;
      d.instance = it->first;
      d.submitted = it->second.submitted;
      d.admitted = it->second.admitted;
      d.finished = now_seconds();
      rc = acopf_poll(s->h, it->first, nullptr, &d.result);
      if (rc) break;
      const int j = d.grid;
      if (s->slots[j] > 0) {
        s->free[j].push_back(s->home[j]);
        s->home[j] = it->first;
      } else {
        s->home_busy[j] = 0;
      }
      s->done.push_back(d);
      it = s->inflight.erase(it);
    }
  }
  if (in_flight) *in_flight = (int32_t)s->inflight.size();
  if (queued) *queued = (int32_t)s->queued;
  return rc;
}

int acopf_server_poll(acopf_server s, acopf_served* out, int32_t max, int32_t* n) {
  if (!s || !n || max < 0 || (max > 0 && !out))
    return fail(ACOPF_EINVAL, "server_poll: null server or output");
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return ACOPF_OK;
}

int acopf_server_info(acopf_server s, int32_t* slots_per_grid, int32_t* home_instance,
                      acopf_result* cold, double* bytes_used, acopf_handle* handle) {
  if (!s) return fail(ACOPF_EINVAL, "null server");
  for (int j = 0; j < s->G; ++j) {
    if (slots_per_grid) slots_per_grid[j] = s->slots[j];
    if (home_instance) home_instance[j] = s->home[j];
    if (cold) cold[j] = s->cold[j];
  }
  if (bytes_used) *bytes_used = s->bytes_used;
  if (handle) *handle = s->h;
  return ACOPF_OK;
}

void acopf_server_destroy(acopf_server s) {
  if (!s) return;
  acopf_destroy(s->h);
  delete s;
}

}  // extern "C"
