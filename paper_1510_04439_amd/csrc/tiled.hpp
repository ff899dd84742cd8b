// Shared declarations of the persistent-queue smoother (smooth_tiled.hip)
// and its callers (the covariance smoother and batched cross-validation).
#pragma once

#include <vector>

#include "common.hpp"

namespace fpca {

constexpr int TQ_THREADS = 512;   // threads per workgroup
constexpr int TQ_SEG = 4;    // consecutive outputs per lane along a pass
constexpr int TQ_MAXX = 14;  // stage-T arrays (d = 3)
constexpr int TQ_MAXY = 27;  // stage-S arrays (d = 3)
constexpr int TQ_NSTAGE = 5;
constexpr int TQ_TILE = 32;   // score tile
constexpr int TQ_MAXSLOT = 3;
constexpr int TQ_CHUNK_MAX = 16;  // queue tasks taken per atomic, at most
constexpr int TQ_SPF = 8;    // stage-S values prefetched per thread
constexpr size_t TQ_LDS_MAX = 160 * 1024 - 256;  // dynamic LDS per workgroup (static LDS is below 256 B)
enum { TQ_T = 0, TQ_S = 1, TQ_W = 2, TQ_SC = 3, TQ_FIN = 4 };

struct TJob {
  const void *Ca, *Cb, *Ga, *Gb;  // C = Ca - Cb, G = Ga - Gb (Cb, Gb may be null)
  const void *Qf, *Gf, *Cf;       // cross-validation: the held-out fold's slabs
  const uint8_t *mask;
  double c0;                      // Ca == null: C = c0 off the diagonal, 0 on it (complete common grid)
  int loo;                        // leave each node's own bin out of its fit (leave-one-out CV)
  void *out;                      // smooth mode: b0, P x P of T
  int8_t *status;                 // smooth mode: optional status
  double h[3];
  int R[3];
  int M[3];
  int P;
  int slot;
  int prev;  // the job that used this slot before, or -1
  int ntask[TQ_NSTAGE];
  int tap_off[3];  // offsets of this job's taps in the launch's tap table
  int pb;    // s-positions per stage-W task
  int tpt;   // score tile pairs per task
};

struct TSeg {
  long long start;
  int job;
  int stage;
};

struct TArgs {
  const TJob *jobs;
  const TSeg *segs;
  int nseg;
  long long total;
  int *qctr;
  int *done;  // [njobs][TQ_NSTAGE]
  int *err;
  double *X[TQ_MAXSLOT];
  double *Y[TQ_MAXSLOT];
  void *Gh[TQ_MAXSLOT];
  double *part;  // [njobs][part_stride]
  int part_stride;
  double *scores;  // [njobs]
  int cv;
  int qb;
  int chunk;  // queue tasks taken per atomic
  const double *taps;  // tap table: per job and coordinate, [e][m + R]
  long long spin_limit;
  int nx, ny;
  const struct TTables *tabs;  // moment bookkeeping of the stages (device copy)
};

// Families, degrees and final-moment indices of the stage-T and stage-S arrays.
struct TTables {
  signed char x_fam[TQ_MAXX], x_deg[TQ_MAXX];
  signed char y_fam[TQ_MAXY], y_deg[TQ_MAXY];
  signed char y_mom[TQ_MAXY][3];
};

// One job: smooth mode (b0 of C = Ca - Cb and G = Ga - Gb into out/status)
// or, in CV mode, the same smooth scored against the held-out fold Qf/Gf/Cf.
struct TiledJob {
  const fpca_grid *grid;
  const void *Ca, *Cb, *Ga, *Gb, *Qf, *Gf, *Cf;
  double c0;  // used when Ca is null
  int loo;    // leave-one-bin-out fit and unsymmetrized score
  const double *h;  // d bandwidths
  void *out;
  int8_t *status;
};

// Tile shape and occupancy of a launch (chosen by the autotuner in CV mode).
struct TiledConfig {
  int qb = 16;         // t-columns per stage-S / stage-W task
  int wg_per_cu = 2;   // persistent workgroups per compute unit
};

struct TiledLaunch {
  TArgs args;
  size_t lds = 0;
  int grid = 0;
  int d = 0;
  bool f64 = false;
  int *zero = nullptr;
  int nzero = 0;
  int njobs = 0;
};

// Grids the engine handles: P <= 4096, and M_1 small enough for the final
// moments of M_1 x QB nodes to sit in LDS.
bool tiled_supported(const fpca_grid *g);
template <typename T>
int tiled_plan(fpca_context *ctx, const std::vector<TiledJob> &jobs, bool cv, const TiledConfig &cfg,
               TiledLaunch *L);
int tiled_queue(fpca_context *ctx, const TiledLaunch &L);
size_t tiled_lds(const std::vector<TiledJob> &jobs, int qb);

}  // namespace fpca
