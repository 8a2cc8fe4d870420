// Autotuner for the register-resident sparse-coding kernels.
//
// For a shape (m1, m2, n1, n2, s) several instantiations exist (how many lanes
// share a signal, split over atom rows and columns, and the register budget
// expressed as waves per SIMD).  sdl_autotune times each on the caller's data with
// HIP events and keeps the fastest for the rest of the process; if the
// environment variable SDL_TUNE_CACHE names a file, choices are read from it on
// first use and appended to it after tuning (one line per shape:
// "m1 m2 n1 n2 s lanes_row lanes_col waves_per_simd matrix_core ms").
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sdl_internal.h"

namespace sdl {
namespace {

using Key = std::tuple<int, int, int, int, int>;
struct Choice {
  int id;
  double ms;
};

std::mutex g_tune_mu;
std::map<Key, Choice> g_choice;
std::map<Key, Choice> g_wave;  // shapes for which the one-wave-per-signal path won (id unused)
// Bumped whenever a kernel choice changes, so captured graphs that baked in the old choice
// are not replayed.
std::atomic<long> g_tune_epoch{0};
bool g_cache_loaded = false;

int find_variant(int m1, int m2, int n1, int n2, int s, int lr, int lc, int wpe, int mfma) {
  int ids[32];
  const int n = omp_fast_variants(m1, m2, n1, n2, s, ids, 32);
  for (int i = 0; i < n && i < 32; ++i) {
    int a, b, c, d;
    omp_fast_variant_info(ids[i], &a, &b, &c, &d);
    if (a == lr && b == lc && c == wpe && d == mfma) return ids[i];
  }
  return -1;
}

void load_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = getenv("SDL_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  int m1, m2, n1, n2, s, lr, lc, wpe, mf;
  double ms;
  while (fscanf(f, "%d %d %d %d %d %d %d %d %d %lf", &m1, &m2, &n1, &n2, &s, &lr, &lc, &wpe, &mf, &ms) == 10) {
    if (mf == 2) {  // one-wave-per-signal path
      g_wave[Key(m1, m2, n1, n2, s)] = Choice{0, ms};
      continue;
    }
    const int id = find_variant(m1, m2, n1, n2, s, lr, lc, wpe, mf);
    if (id >= 0) {
      g_choice[Key(m1, m2, n1, n2, s)] = Choice{id, ms};
      g_wave.erase(Key(m1, m2, n1, n2, s));
    }
  }
  fclose(f);
}

void append_cache(const Key& k, int id, double ms) {
  const char* path = getenv("SDL_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  int lr, lc, wpe, mf;
  omp_fast_variant_info(id, &lr, &lc, &wpe, &mf);
  fprintf(f, "%d %d %d %d %d %d %d %d %d %.6f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
          std::get<4>(k), lr, lc, wpe, mf, ms);
  fclose(f);
}

}  // namespace

long tuning_epoch() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  return g_tune_epoch.load();
}

int omp_fast_choice(int m1, int m2, int n1, int n2, int s) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  auto it = g_choice.find(Key(m1, m2, n1, n2, s));
  if (it != g_choice.end()) return it->second.id;
  int id = -1;
  omp_fast_variants(m1, m2, n1, n2, s, &id, 1);
  return id;
}

void omp_fast_set_choice(int m1, int m2, int n1, int n2, int s, int id) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_choice[Key(m1, m2, n1, n2, s)] = Choice{id, 0.0};
  ++g_tune_epoch;
}

bool wave_chosen(int m1, int m2, int n1, int n2, int s) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  return g_wave.count(Key(m1, m2, n1, n2, s)) > 0;
}

double wave_choice_ms(int m1, int m2, int n1, int n2, int s) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_wave.find(Key(m1, m2, n1, n2, s));
  return it == g_wave.end() ? 0.0 : it->second.ms;
}

void set_wave_choice(int m1, int m2, int n1, int n2, int s, bool on, double ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  const Key k(m1, m2, n1, n2, s);
  ++g_tune_epoch;
  if (!on) {
    g_wave.erase(k);
    return;
  }
  g_wave[k] = Choice{0, ms};
  int lr = 0, lc = 0;
  if (ms > 0.0 && omp_wave_grid(m1, m2, n1, n2, s, &lr, &lc)) {
    const char* path = getenv("SDL_TUNE_CACHE");
    if (path && *path) {
      FILE* f = fopen(path, "a");
      if (f) {
        fprintf(f, "%d %d %d %d %d %d %d %d %d %.6f\n", m1, m2, n1, n2, s, lr, lc, 0, 2, ms);
        fclose(f);
      }
    }
  }
}

// Times every variant of one problem's shape; returns hipSuccess and the chosen id/ms.
hipError_t autotune_problem(const OmpArgs<float>& a, hipStream_t st, int reps, int* chosen, double* best_ms) {
  int ids[32];
  const int n = std::min(32, omp_fast_variants(a.m1, a.m2, a.n1, a.n2, a.s, ids, 32));
  *chosen = -1;
  *best_ms = 0.0;
  if (n == 0 || a.N == 0) return hipSuccess;
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) return err;
  double best = 1e300;
  int best_id = ids[0];
  for (int i = 0; i < n && err == hipSuccess; ++i) {
    err = launch_omp_fast_variant(ids[i], a, st);  // warm-up
    if (err != hipSuccess) break;
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
      if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
      if ((err = launch_omp_fast_variant(ids[i], a, st)) != hipSuccess) break;
      if ((err = hipEventRecord(e1, st)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      t.push_back(ms);
    }
    if (err != hipSuccess || t.empty()) break;
    std::sort(t.begin(), t.end());
    const double med = t[t.size() / 2];
    if (med < best) {
      best = med;
      best_id = ids[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return err;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    const Key k(a.m1, a.m2, a.n1, a.n2, a.s);
    g_choice[k] = Choice{best_id, best};
    ++g_tune_epoch;
    append_cache(k, best_id, best);
  }
  *chosen = best_id;
  *best_ms = best;
  return hipSuccess;
}

bool tuned_config(int m1, int m2, int n1, int n2, int s, int* lr, int* lc, int* wpe, int* mfma, double* ms) {
  int id;
  double t = 0.0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_choice.find(Key(m1, m2, n1, n2, s));
    if (it != g_choice.end()) {
      id = it->second.id;
      t = it->second.ms;
    } else {
      id = -1;
      omp_fast_variants(m1, m2, n1, n2, s, &id, 1);
    }
  }
  if (id < 0) return false;
  omp_fast_variant_info(id, lr, lc, wpe, mfma);
  if (ms) *ms = t;
  return true;
}

}  // namespace sdl
