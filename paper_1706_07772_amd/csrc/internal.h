// Host-side internals shared by the library's translation units.
#pragma once

#include "reaxff_dev.h"

namespace rx {

// scratch owned by the context (device pointers)
struct Scratch {
  int32_t* cid = nullptr;         // [n] cell of each caller-order atom
  int32_t* cell_s = nullptr;      // [n] cell of each sorted atom
  int32_t* cell_count = nullptr;  // [ncell + 1]
  int32_t* cell_cursor = nullptr; // [ncell + 1]
  int32_t* flag = nullptr;        // error flags written by kernels
  int32_t* cnt_far = nullptr;     // [n + 1]
  int32_t* cnt_bond = nullptr;    // [n + 1]
  int32_t* cnt_hb = nullptr;      // [n + 1]
  double* part = nullptr;         // bbox partials
  int64_t* totals = nullptr;      // device [4]
  int64_t* totals_host = nullptr; // pinned host [4]
  // scan temporaries
  int64_t* scan_tmp = nullptr;
  int64_t scan_cap = 0;
};

// exclusive prefix sums; out[n-1] holds the total when in[n-1] == 0
int scan_i32(const int32_t* in, int32_t* out, int64_t n, Scratch& sc, hipStream_t st);
int scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Scratch& sc, hipStream_t st);

int launch_bbox(const double* pos, const int32_t* type, int64_t n, double* part, int nparts,
                int32_t* flag, hipStream_t st);
int launch_cell_sort(const double* pos, const int32_t* type, int64_t n, const Grid& g, int ncell,
                     Scratch& sc, Lists& L, hipStream_t st);
int launch_count(const DevParams* P, const Grid& g, int64_t n, Scratch& sc, Lists& L, hipStream_t st);
int launch_fill(const DevParams* P, const Grid& g, int64_t n, Scratch& sc, Lists& L, hipStream_t st);
int launch_export(const Lists& L, int32_t* far, int32_t* bonds, int32_t* hb, hipStream_t st);

int launch_forces(const DevParams* P, const Grid& g, const Lists& L, Work& W, const double* q,
                  double* forces, double* energies, hipStream_t st);
int launch_kick(int64_t n, double* vel, const double* forces, const int32_t* type,
                const DevParams* P, double half_dt, hipStream_t st);
int launch_drift(int64_t n, double* pos, const double* vel, double dt, const Grid& g, hipStream_t st);
int launch_kinetic(int64_t n, const double* vel, const int32_t* type, const DevParams* P,
                   double* out, hipStream_t st);

}  // namespace rx
