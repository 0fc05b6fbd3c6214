// Served requests: a pool of independent solves that share one GPU.
//
// Each admitted request is its own solver handle on one of a few HIP
// streams (all at the default priority), so requests that arrive while
// others run are admitted as soon as their device footprint fits in the
// budget, and their kernels overlap on the device.  A tick enqueues up to k
// steps for every running request, then waits; finished requests keep their
// results until collected.  All pool calls are thread-safe: a host thread
// may admit (and build the mesh of) a new request while another launches and
// collects steps; the mesh build runs outside the pool lock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_internal.hpp"

namespace {
thread_local std::string g_pool_err;
}

extern "C" const char *fr_last_error(void);

struct fr_pool {
  std::mutex mu;
  size_t budget = 0, used = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  struct Req {
    fr_mesh *m = nullptr;
    int64_t left = 0, total = 0;
    size_t bytes = 0;
    bool done = false, in_flight = false;
    fr_status status = FR_OK;
    // data surface (sampled requests): snapshot j is taken after warmup + j * every steps
    fr_probe *probe = nullptr;
    fr_fwh *rec = nullptr;
    int64_t warmup = 0, every = 1, n_samples = 0, taken = 0;
    int64_t next_sample() const { return taken < n_samples ? warmup + taken * every : -1; }
    void release() {
      fr_probe_destroy(probe);
      fr_fwh_destroy(rec);
      fr_mesh_destroy(m);
      probe = nullptr;
      rec = nullptr;
      m = nullptr;
    }
  };
  std::map<int64_t, Req> reqs;
  int64_t next_slot = 0, rr = 0;
};

extern "C" {

fr_status fr_footprint(const fr_mesh_desc *d, size_t *bytes) {
  if (!d || !bytes || d->n_elems <= 0 || (d->dim != 2 && d->dim != 3)) return FR_E_ARG;
  if (d->elem_order) {
    // variable order: the order groups' footprints, plus the mortar data for at most
    // every face point of every element
    size_t total = 0;
    std::vector<int64_t> en_count(8, 0);
    for (int64_t e = 0; e < d->n_elems; ++e) {
      const int p = d->elem_order[e];
      if (p < 0 || p > 7) return FR_E_ARG;
      ++en_count[size_t(p)];
    }
    for (int p = 0; p < 8; ++p) {
      if (!en_count[size_t(p)]) continue;
      fr_mesh_desc g = *d;
      g.elem_order = nullptr;
      g.order = p;
      g.n_elems = en_count[size_t(p)];
      g.n_bfaces = 0;
      size_t b = 0;
      const fr_status st = fr_footprint(&g, &b);
      if (st != FR_OK) return st;
      total += b;
    }
    int64_t nwall = 0, maxp = 1;
    for (int64_t e = 0; e < d->n_elems; ++e) maxp = std::max<int64_t>(maxp, d->elem_order[e]);
    for (int64_t i = 0; i < d->n_bfaces; ++i)
      if (d->bfaces[3 * i + 2] == FR_BC_WALL) ++nwall;
    const fr::Dims D(d->dim, int(maxp));
    const size_t rs = d->precision == FR_FP32 ? 4 : 8;
    total += size_t(nwall) * D.nfp * 3 * 8;
    if (d->dim == 3)  // column metrics of groups of extruded elements, at the highest order
      total += size_t(d->n_elems + 8 * fr::EB) * 8 *
               (size_t(D.n) * D.n * 4 + D.n + (4 * size_t(D.n) + size_t(D.n) * D.n) * 2 + size_t(D.n) * D.n + D.n);
    // mortar data. Faces are matched by their corner node ids; a face shared by elements
    // of two orders carries nfp_H + nfp_L mortar points, nfp_H nfp_L interpolation entries
    // and, for its lower-order points, nfp_L nfp_H trace and nfp_L nfp_H projection
    // entries. A face matched by no other element and not a listed boundary face (a
    // periodic face, paired by translation) is counted as a mortar face at the highest
    // order on both sides, an upper bound.
    const int dim = d->dim, q = d->geom_order, na = q + 1, nfe = 2 * dim, nc = dim == 2 ? 2 : 4;
    const int nn = dim == 2 ? na * na : na * na * na;
    if (q < 1 || !d->nodes || !d->elem_nodes) return FR_E_ARG;
    auto nfp_of = [&](int64_t p) { return size_t(dim == 2 ? p + 1 : (p + 1) * (p + 1)); };
    std::set<std::pair<int64_t, int>> listed;
    for (int64_t i = 0; i < d->n_bfaces; ++i) listed.insert({d->bfaces[3 * i], int(d->bfaces[3 * i + 1])});
    std::map<std::array<int64_t, 4>, std::pair<int64_t, int>> seen;  // corner ids -> (element, face)
    size_t mpts = 0, ment = 0, pent = 0;
    auto add = [&](size_t hi, size_t lo) {
      mpts += hi + lo;
      ment += 2 * hi * lo;
      pent += hi * lo;
    };
    for (int64_t e = 0; e < d->n_elems; ++e)
      for (int f = 0; f < nfe; ++f) {
        const int k = f / 2;
        std::array<int64_t, 4> key{-1, -1, -1, -1};
        for (int c = 0; c < nc; ++c) {
          int a[3] = {0, 0, 0}, o = 0;
          a[k] = (f & 1) * q;
          for (int j = 0; j < dim; ++j)
            if (j != k) a[j] = ((c >> o++) & 1) * q;
          key[size_t(c)] = d->elem_nodes[e * nn + a[0] + na * a[1] + na * na * a[2]];
        }
        std::sort(key.begin(), key.begin() + nc);
        auto it = seen.find(key);
        if (it == seen.end()) {
          seen.emplace(key, std::make_pair(e, f));
          continue;
        }
        const int64_t pa = d->elem_order[it->second.first], pb = d->elem_order[e];
        if (pa != pb) add(nfp_of(std::max(pa, pb)), nfp_of(std::min(pa, pb)));
        seen.erase(it);
      }
    for (const auto &kv : seen)
      if (!listed.count(kv.second)) add(D.nfp, D.nfp);
    // MT, the two per-point offset tables, the trace / half-flux entries (group, code,
    // weight) and the projection entries (code, weight), and the groups' pointer arrays
    total += std::max<size_t>(mpts, 1) * D.nv * rs + (mpts + 2) * (2 * 4) + ment * (4 + 4 + 8) +
             pent * (4 + 8) + 4 * 256;
    *bytes = total;
    return FR_OK;
  }
  if (d->order < 0) return FR_E_ARG;
  const fr::Dims D(d->dim, d->order);
  const size_t rs = d->precision == FR_FP32 ? 4 : 8;
  const int64_t nblk = (d->n_elems + fr::EB - 1) / fr::EB;
  int64_t nwall = 0;
  for (int64_t i = 0; i < d->n_bfaces; ++i)
    if (d->bfaces[3 * i + 2] == FR_BC_WALL) nwall += D.nfp;
  auto r256 = [](size_t n) { return n == 0 ? size_t(256) : n; };
  const int dim = d->dim, nv = D.nv;
  const int RTU = D.nup / 16, RTF = D.nfpad / 16, KTU = D.ku / 4, KTF = D.kf / 4;
  size_t b = 0;
  // operators
  b += r256(size_t(RTF) * KTU * 64 * rs) + r256(size_t(dim) * RTU * KTU * 64 * rs) +
       r256(size_t(dim) * RTU * KTF * 64 * rs) + r256(size_t(RTU) * dim * KTU * 64 * rs) +
       r256(size_t(RTU) * KTF * 64 * rs) + r256(size_t(2 * D.n * D.n + 4 * D.n) * rs);
  // geometry and tables
  b += size_t(nblk) * D.nup * dim * dim * fr::EB * 8 + size_t(nblk) * D.nup * fr::EB * 8;
  b += size_t(nblk) * D.nfpad * dim * fr::EB * 8 + size_t(nblk) * D.nfpad * fr::EB * 8;
  b += size_t(nblk) * D.nfpad * fr::EB * 4 + size_t(nblk) * 2 * dim * fr::EB * 4;  // per-point and per-face codes
  if (dim == 3) b += size_t(nblk) * 27 * 3 * fr::EB * 8 + size_t(6 * D.n) * 8;  // geometry nodes, basis
  if (fr::desc_extruded(*d))  // column metrics and the reciprocal column and layer factors of |J|
    b += size_t(nblk) * fr::EB * 8 *
         (size_t(D.n) * D.n * 4 + D.n + (4 * size_t(D.n) + size_t(D.n) * D.n) * 2 + size_t(D.n) * D.n + D.n);
  b += r256(nblk * 4) * 2 + r256(nblk * 8) * 2 + r256(5 * 8) + r256(2 * 8) + r256(D.nfpad * 8);
  // state and stage arrays
  const size_t nU = size_t(nblk) * D.nup * nv * fr::EB, nF = size_t(nblk) * D.nfpad * nv * fr::EB;
  const size_t nG = size_t(nblk) * D.nup * dim * nv * fr::EB;
  b += 4 * nU * rs + 4 * nF * rs + 2 * nG * rs;
  b += r256(size_t(std::max<int64_t>(nwall, 1)) * 3 * 8) + r256(8 * 8) + r256(4);
  b += size_t(d->n_elems) * D.nu * nv * 8;
  *bytes = b;
  return FR_OK;
}

fr_status fr_pool_create(size_t budget, int32_t device, fr_pool **out) {
  if (!out || budget == 0) return FR_E_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return FR_E_DEVICE;
  fr_pool *p = new fr_pool();
  p->budget = budget;
  p->device = device;
  for (int i = 0; i < 4; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto t : p->streams) (void)hipStreamDestroy(t);
      delete p;
      return FR_E_DEVICE;
    }
    p->streams.push_back(s);
  }
  *out = p;
  return FR_OK;
}

void fr_pool_destroy(fr_pool *p) {
  if (!p) return;
  for (auto &kv : p->reqs) kv.second.release();
  for (auto s : p->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  delete p;
}

}  // extern "C"

namespace {

bool valid_surface(const fr_pool_surface *s) {
  return s->n_points > 0 && s->points && s->normals && s->areas && s->n_copies >= 1 && s->warmup >= 0 &&
         s->every >= 1 && s->n_samples >= 8;
}

fr_status admit(fr_pool *p, const fr_mesh_desc *desc, const double *u0, int64_t steps, const fr_pool_surface *surf,
                int64_t *slot) {
  size_t need = 0;
  fr_status st = fr_footprint(desc, &need);
  if (st != FR_OK) return st;
  if (surf)
    need += fr::probe_footprint(surf->n_points, desc->dim, desc->order) +
            fr::fwh_footprint(surf->n_points, surf->n_samples);
  hipStream_t stream;
  {
    // reserve the footprint first so that concurrent admissions respect the budget
    std::lock_guard<std::mutex> lk(p->mu);
    if (need > p->budget - std::min(p->budget, p->used)) return FR_E_NOMEM;
    p->used += need;
    stream = p->streams[p->rr++ % p->streams.size()];
  }
  fr_pool::Req r;
  auto undo = [&](fr_status code) {
    r.release();
    std::lock_guard<std::mutex> lk(p->mu);
    p->used -= std::min(p->used, need);
    return code;
  };
  fr_mesh_desc d = *desc;
  d.device = p->device;
  d.stream = stream;
  st = fr_mesh_create(&d, &r.m);
  if (st != FR_OK) return undo(st);
  int64_t info[10], npts = 0;
  fr_mesh_info(r.m, info);
  fr_mesh_points(r.m, &npts);
  const int64_t n = npts * info[6];
  std::vector<double> u;
  if (!u0) {
    u.resize(size_t(n));
    const int dim = desc->dim;
    const double *fs = desc->freestream;
    double ke = 0.0;
    for (int k = 0; k < dim; ++k) ke += fs[1 + k] * fs[1 + k];
    for (int64_t i = 0; i < n / (dim + 2); ++i) {
      double *x = &u[size_t(i) * (dim + 2)];
      x[0] = fs[0];
      for (int k = 0; k < dim; ++k) x[1 + k] = fs[0] * fs[1 + k];
      x[dim + 1] = fs[4] / (desc->gamma - 1.0) + 0.5 * fs[0] * ke;
    }
    u0 = u.data();
  }
  st = fr_set_state(r.m, u0);
  if (st != FR_OK) return undo(st);
  if (surf) {
    st = fr_probe_create(r.m, &d, 0, surf->n_points, surf->points, &r.probe);
    if (st != FR_OK) return undo(st);
    const double *fs = desc->freestream;
    fr_fwh_desc fd{};
    fd.n_points = surf->n_points;
    fd.points = surf->points;
    fd.normals = surf->normals;
    fd.areas = surf->areas;
    fd.n_copies = surf->n_copies;
    fd.c0 = std::sqrt(desc->gamma * fs[4] / fs[0]);
    for (int i = 0; i < 3; ++i) {
      fd.copy_shift[i] = surf->copy_shift[i];
      fd.mach[i] = (i < desc->dim ? fs[1 + i] : 0.0) / fd.c0;
    }
    fd.rho0 = fs[0];
    fd.p0 = fs[4];
    fd.dt = double(surf->every) * desc->dt;
    fd.tau0 = 0.0;
    fd.capacity = surf->n_samples;
    fd.device = p->device;
    fd.stream = stream;
    st = fr_fwh_create(&fd, &r.rec);
    if (st != FR_OK) return undo(st);
    r.warmup = surf->warmup;
    r.every = surf->every;
    r.n_samples = surf->n_samples;
  }
  r.left = r.total = steps;
  r.bytes = need;
  std::lock_guard<std::mutex> lk(p->mu);
  *slot = p->next_slot++;
  p->reqs[*slot] = r;
  return FR_OK;
}

// Enqueue up to k steps of a running request, with its due snapshots in between.
fr_status enqueue(fr_pool::Req &r, int64_t k) {
  bool first = true;
  for (;;) {
    const int64_t pos = r.total - r.left;
    if (r.next_sample() == pos) {
      fr_status st = FR_OK;
      if (r.taken == 0) st = fr::means_clear(r.m);  // means over the sampled period
      if (st == FR_OK) st = fr::fwh_append_probe_async(r.rec, r.probe);
      if (st != FR_OK) return st;
      ++r.taken;
      continue;
    }
    if (k == 0 || r.left == 0) return FR_OK;
    int64_t n = std::min(k, r.left);
    if (r.next_sample() > pos) n = std::min(n, r.next_sample() - pos);
    const fr_status st = fr::step_enqueue(r.m, n, first);
    if (st != FR_OK) return st;
    first = false;
    r.left -= n;
    k -= n;
  }
}

}  // namespace

extern "C" {

fr_status fr_pool_admit(fr_pool *p, const fr_mesh_desc *desc, const double *u0, int64_t steps, int64_t *slot) {
  if (!p || !desc || !slot || steps <= 0) return FR_E_ARG;
  return admit(p, desc, u0, steps, nullptr, slot);
}

fr_status fr_pool_admit_sampled(fr_pool *p, const fr_mesh_desc *desc, const double *u0, const fr_pool_surface *s,
                                int64_t *slot) {
  if (!p || !desc || !slot || !s || !valid_surface(s)) return FR_E_ARG;
  return admit(p, desc, u0, s->warmup + (s->n_samples - 1) * s->every, s, slot);
}

fr_status fr_pool_launch(fr_pool *p, int64_t k) {
  if (!p || k <= 0) return FR_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  for (auto &kv : p->reqs) {
    auto &r = kv.second;
    if (r.done || r.in_flight) continue;
    const fr_status st = enqueue(r, k);
    r.in_flight = true;  // collect waits for what was enqueued, also after a failure
    if (st != FR_OK) {
      r.done = true;
      r.status = st;
    }
  }
  return FR_OK;
}

fr_status fr_pool_collect(fr_pool *p, int64_t *done, int32_t max_done, int32_t *n_done) {
  if (!p || !n_done) return FR_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  *n_done = 0;
  for (auto &kv : p->reqs) {
    auto &r = kv.second;
    if (!r.in_flight) {
      if (r.done && r.status != FR_OK && done && *n_done < max_done) done[(*n_done)++] = kv.first;
      continue;
    }
    r.in_flight = false;
    const fr_status st = fr_sync(r.m);
    if (r.status == FR_OK && st != FR_OK) {
      r.done = true;
      r.status = st;
    } else if (r.left == 0 && r.next_sample() < 0) {
      r.done = true;
    }
    if (r.done && done && *n_done < max_done) done[(*n_done)++] = kv.first;
  }
  return FR_OK;
}

fr_status fr_pool_tick(fr_pool *p, int64_t k, int64_t *done, int32_t max_done, int32_t *n_done) {
  const fr_status st = fr_pool_launch(p, k);
  if (st != FR_OK) return st;
  return fr_pool_collect(p, done, max_done, n_done);
}

fr_status fr_pool_result(fr_pool *p, int64_t slot, double *out, double *u) {
  if (!p) return FR_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->reqs.find(slot);
  if (it == p->reqs.end()) return FR_E_ARG;
  auto &r = it->second;
  if (!r.done || r.in_flight) return FR_E_STATE;
  fr_status st = r.status;
  if (st == FR_OK && out) st = fr_forces(r.m, 0, out);
  if (st == FR_OK && u) st = fr_get_state(r.m, u);
  r.release();
  p->used -= std::min(p->used, r.bytes);
  p->reqs.erase(it);
  return st;
}

fr_status fr_pool_pressure(fr_pool *p, int64_t slot, const double *observer, int64_t capacity, double *t_start,
                           int64_t *n_out, double *pressure) {
  if (!p || !observer || !t_start || !n_out || !pressure) return FR_E_ARG;
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->reqs.find(slot);
  if (it == p->reqs.end()) return FR_E_ARG;
  auto &r = it->second;
  if (!r.done || r.in_flight || r.status != FR_OK || !r.rec) return FR_E_STATE;
  return fr_fwh_pressure(r.rec, observer, capacity, t_start, n_out, pressure, nullptr, nullptr);
}

fr_status fr_pool_usage(const fr_pool *p, int64_t *used) {
  if (!p || !used) return FR_E_ARG;
  std::lock_guard<std::mutex> lk(const_cast<fr_pool *>(p)->mu);
  used[0] = int64_t(p->used);
  int64_t running = 0;
  for (auto &kv : p->reqs)
    if (!kv.second.done) ++running;
  used[1] = running;
  return FR_OK;
}

}  // extern "C"
