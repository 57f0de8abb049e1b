// Batched execution of many independent realisations of uneven size
// (HOS steps + interpolation to each realisation's cells) as one hipGraph
// launch.  The realisations' launch chains are captured as parallel branches
// over K worker streams (fork/join through events), so kernels of different
// realisations overlap on the GPU; K is chosen by timing candidates with HIP
// events (autotune) and cached on disk keyed by (architecture, batch shape).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

struct swense_batch {
  std::vector<swense_hos*> hos;
  std::vector<swense_cells*> cells;
  std::vector<unsigned> masks;
  std::vector<float*> outs;
  int nsteps = 1;
  hipStream_t st = nullptr;          // launch stream (may be the null stream)
  hipStream_t cap = nullptr;         // capture origin (never the null stream)
  std::vector<hipStream_t> workers;  // capture branches
  std::vector<hipEvent_t> evs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int k = 0;  // branches of the current graph
  std::vector<long> epochs;  // each realisation's scratch epoch when the graph was captured
  std::string err;
  std::string signature;
};

namespace {

void release_graph(swense_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void ensure_workers(swense_batch* b, int k) {
  while ((int)b->workers.size() < k) {
    hipStream_t s;
    SW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->workers.push_back(s);
  }
  while ((int)b->evs.size() < 2 * k + 1) {
    hipEvent_t e;
    SW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->evs.push_back(e);
  }
}

// The work of realisation i on its handle's current stream.
void enqueue_one(swense_batch* b, int i) {
  swense_hos* h = b->hos[i];
  int rc = swense_hos_step(h, b->nsteps);
  if (rc != SWENSE_OK) throw SwenseError{rc, std::string("batch step: ") + h->err};
  if (b->cells[i]) {
    rc = swense_interp_cells(h, b->cells[i], b->masks[i], b->outs[i], nullptr);
    if (rc != SWENSE_OK) throw SwenseError{rc, std::string("batch interp: ") + h->err};
  }
}

// Capture every realisation as a branch: branch j runs realisations j, j+K, ...
void capture(swense_batch* b, int k) {
  release_graph(b);
  ensure_workers(b, k);
  // capturing runs the host side of every call once: keep streams and times
  std::vector<hipStream_t> saved(b->hos.size());
  std::vector<double> t0(b->hos.size());
  for (size_t i = 0; i < b->hos.size(); ++i) {
    saved[i] = b->hos[i]->st;
    t0[i] = b->hos[i]->t;
  }
  auto put_back = [&]() {
    for (size_t i = 0; i < b->hos.size(); ++i) {
      b->hos[i]->st = saved[i];
      b->hos[i]->t = t0[i];
      b->hos[i]->version++;
    }
  };
  if (!b->cap) SW_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  SW_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  try {
    SW_HIP(hipEventRecord(b->evs[0], b->cap));
    for (int j = 0; j < k; ++j) SW_HIP(hipStreamWaitEvent(b->workers[j], b->evs[0], 0));
    for (size_t i = 0; i < b->hos.size(); ++i) {
      b->hos[i]->st = b->workers[i % k];
      // with cells, each replay ends with the modes (and right-hand side) of
      // the new state, so the next replay's first RK stage may take it
      b->hos[i]->graph_reuse_k = b->cells[i] != nullptr;
      enqueue_one(b, (int)i);
      b->hos[i]->graph_reuse_k = false;
    }
    for (int j = 0; j < k; ++j) {
      SW_HIP(hipEventRecord(b->evs[1 + j], b->workers[j]));
      SW_HIP(hipStreamWaitEvent(b->cap, b->evs[1 + j], 0));
    }
  } catch (...) {
    for (swense_hos* h : b->hos) h->graph_reuse_k = false;
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    put_back();
    throw;
  }
  put_back();
  SW_HIP(hipStreamEndCapture(b->cap, &b->graph));
  SW_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->k = k;
  b->epochs.clear();
  for (swense_hos* h : b->hos) b->epochs.push_back(h->scratch_epoch);
}

// Host bookkeeping after the graph ran once: every realisation advanced.
void advance_host(swense_batch* b) {
  for (size_t i = 0; i < b->hos.size(); ++i) {
    swense_hos* h = b->hos[i];
    h->t += b->nsteps * h->d.dt;
    h->version++;
    if (b->cells[i]) {
      // the graph recomputed the modes and the right-hand side last
      h->modes_version = h->version;
      h->kk_version = h->version;
    }
  }
}

// Before a launch: the first RK stage of realisations with cells takes the
// right-hand side of the current state, so evaluate it where it is stale.
void prime(swense_batch* b) {
  bool any = false;
  for (size_t i = 0; i < b->hos.size(); ++i) {
    swense_hos* h = b->hos[i];
    if (b->cells[i] && h->kk_version != h->version) {
      hos_prime_rhs(h);
      any = true;
    }
  }
  if (!any) return;
  for (size_t i = 0; i < b->hos.size(); ++i)
    if (b->cells[i]) SW_HIP(hipStreamSynchronize(b->hos[i]->st));
}

struct Saved {
  std::vector<std::vector<cd>> e, p;
  std::vector<double> t;
};

Saved save_states(swense_batch* b) {
  Saved s;
  for (swense_hos* h : b->hos) {
    std::vector<cd> e(h->nc), p(h->nc);
    SW_HIP(hipMemcpy(e.data(), h->xn[0], h->nc * sizeof(cd), hipMemcpyDeviceToHost));
    SW_HIP(hipMemcpy(p.data(), h->xn[1], h->nc * sizeof(cd), hipMemcpyDeviceToHost));
    s.e.push_back(std::move(e));
    s.p.push_back(std::move(p));
    s.t.push_back(h->t);
  }
  return s;
}

void restore_states(swense_batch* b, const Saved& s) {
  for (size_t i = 0; i < b->hos.size(); ++i) {
    swense_hos* h = b->hos[i];
    SW_HIP(hipMemcpy(h->xn[0], s.e[i].data(), h->nc * sizeof(cd), hipMemcpyHostToDevice));
    SW_HIP(hipMemcpy(h->xn[1], s.p[i].data(), h->nc * sizeof(cd), hipMemcpyHostToDevice));
    h->t = s.t[i];
    h->version++;
  }
}

double time_graph(swense_batch* b, int reps) {
  hipEvent_t e0, e1;
  SW_HIP(hipEventCreate(&e0));
  SW_HIP(hipEventCreate(&e1));
  prime(b);
  SW_HIP(hipGraphLaunch(b->exec, b->st));  // warm
  SW_HIP(hipEventRecord(e0, b->st));
  for (int r = 0; r < reps; ++r) SW_HIP(hipGraphLaunch(b->exec, b->st));
  SW_HIP(hipEventRecord(e1, b->st));
  SW_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  SW_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName);
}

// cache file: one JSON object {"key": k, ...}, read and rewritten whole
bool cache_lookup(const std::string& path, const std::string& key, int* k) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  const std::string q = "\"" + key + "\"";
  size_t pos = s.find(q);
  if (pos == std::string::npos) return false;
  pos = s.find(':', pos + q.size());
  if (pos == std::string::npos) return false;
  *k = std::atoi(s.c_str() + pos + 1);
  return *k > 0;
}

void cache_store(const std::string& path, const std::string& key, int k) {
  std::string s;
  {
    std::ifstream f(path);
    if (f) {
      std::stringstream ss;
      ss << f.rdbuf();
      s = ss.str();
    }
  }
  std::vector<std::pair<std::string, int>> entries;
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    std::string kk = s.substr(pos + 1, end - pos - 1);
    size_t colon = s.find(':', end);
    if (colon == std::string::npos) break;
    entries.emplace_back(kk, std::atoi(s.c_str() + colon + 1));
    pos = s.find_first_of(",}", colon);
    if (pos == std::string::npos) break;
  }
  bool found = false;
  for (auto& e : entries)
    if (e.first == key) {
      e.second = k;
      found = true;
    }
  if (!found) entries.emplace_back(key, k);
  std::ofstream o(path, std::ios::trunc);
  o << "{\n";
  for (size_t i = 0; i < entries.size(); ++i)
    o << "  \"" << entries[i].first << "\": " << entries[i].second << (i + 1 < entries.size() ? ",\n" : "\n");
  o << "}\n";
}

int guarded_b(swense_batch* b, const std::function<int()>& f) {
  try {
    return f();
  } catch (const SwenseError& e) {
    if (b) b->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (b) b->err = e.what();
    return SWENSE_EHIP;
  }
}

}  // namespace

extern "C" {

int swense_batch_create(swense_hos* const* hos, swense_cells* const* cells, const unsigned* masks,
                        float* const* outs, int n, int nsteps, void* stream, swense_batch** out) {
  if (!out || !hos || n <= 0 || nsteps < 1) return SWENSE_EINVAL;
  *out = nullptr;
  swense_batch* b = new swense_batch();
  int rc = guarded_b(b, [&] {
    b->st = reinterpret_cast<hipStream_t>(stream);
    b->nsteps = nsteps;
    std::ostringstream sig;
    sig << "n" << n << "s" << nsteps;
    for (int i = 0; i < n; ++i) {
      SW_REQUIRE(hos[i] != nullptr, "null realisation handle");
      b->hos.push_back(hos[i]);
      swense_cells* c = cells ? cells[i] : nullptr;
      b->cells.push_back(c);
      b->masks.push_back(c ? (masks ? masks[i] : (unsigned)SWENSE_ALL_FIELDS) : 0u);
      SW_REQUIRE(!c || (outs && outs[i]), "interpolating realisation without an output buffer");
      b->outs.push_back(c ? outs[i] : nullptr);
      sig << "_" << hos[i]->G.nx << "x" << hos[i]->G.ny << "m" << hos[i]->d.order_m;
    }
    b->signature = sig.str();
    // eager warm-up with the states restored afterwards: allocates every
    // workspace and sets kernel attributes outside the capture
    Saved s = save_states(b);
    for (int i = 0; i < n; ++i) enqueue_one(b, i);
    for (swense_hos* h : b->hos) SW_HIP(hipStreamSynchronize(h->st));
    restore_states(b, s);
    capture(b, std::min(n, 8));
    return (int)SWENSE_OK;
  });
  if (rc != SWENSE_OK) {
    swense_batch_destroy(b);
    return rc;
  }
  *out = b;
  return SWENSE_OK;
}

int swense_batch_run(swense_batch* b) {
  if (!b || !b->exec) return SWENSE_EINVAL;
  return guarded_b(b, [&] {
    // a call outside the graph reallocated a buffer the graph writes (a larger
    // evaluation, mask or window since the capture): capture again, which
    // records the new addresses (buffers only grow, so nothing is allocated
    // while capturing)
    bool stale = b->epochs.size() != b->hos.size();
    for (size_t i = 0; i < b->hos.size() && !stale; ++i) stale = b->hos[i]->scratch_epoch != b->epochs[i];
    if (stale) capture(b, b->k);
    prime(b);
    SW_HIP(hipGraphLaunch(b->exec, b->st));
    advance_host(b);
    return (int)SWENSE_OK;
  });
}

int swense_batch_autotune(swense_batch* b, const char* cache_path, int* chosen, double* best_ms) {
  if (!b) return SWENSE_EINVAL;
  return guarded_b(b, [&] {
    const std::string key = arch_name() + "|batch|" + b->signature;
    int k = 0;
    if (cache_path && cache_lookup(cache_path, key, &k)) {
      if (k != b->k) capture(b, std::min<int>(k, (int)b->hos.size()));
      if (chosen) *chosen = b->k;
      if (best_ms) *best_ms = -1.0;
      return (int)SWENSE_OK;
    }
    Saved s = save_states(b);
    const int n = (int)b->hos.size();
    double best = 1e300;
    int bestk = 1;
    for (int cand : {1, 2, 4, 8, 16, 32, 64}) {
      if (cand > n) break;
      capture(b, cand);
      const double ms = time_graph(b, 3);
      if (ms < best) {
        best = ms;
        bestk = cand;
      }
    }
    capture(b, bestk);
    restore_states(b, s);
    if (cache_path) cache_store(cache_path, key, bestk);
    if (chosen) *chosen = bestk;
    if (best_ms) *best_ms = best;
    return (int)SWENSE_OK;
  });
}

const char* swense_batch_last_error(const swense_batch* b) { return b ? b->err.c_str() : "no batch"; }

void swense_batch_destroy(swense_batch* b) {
  if (!b) return;
  release_graph(b);
  for (auto s : b->workers) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto e : b->evs) (void)hipEventDestroy(e);
  delete b;
}

}  // extern "C"
