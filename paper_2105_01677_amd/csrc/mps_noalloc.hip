// Allocation-free neighbour search: the cell sort (a1) and the neighbour
// lists (a2) of mps_neighbors for positions the caller passes, with every
// work array carved out of one fixed device array instead of a context's
// allocations.  For callers that cannot allocate device memory (code under
// stream capture, serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is a file-scope __device__ variable: each GPU
// the library runs on holds its own copy, at its own address, until the
// process ends.  Host code never passes the symbol itself to a kernel (on
// the host it is only a stand-in, not a device address): the device address
// is looked up once per device with hipGetSymbolAddress and kept.  Every
// call on one GPU shares that GPU's copy and leaves the last call's data in
// it, so the parts that must start at zero (the cell counts and the status
// word) are cleared by a fill kernel at each call, and calls that overlap on
// one GPU (different streams or threads) race.
#include <cstdio>
#include <cstring>
#include <mutex>

#include "mps_internal.h"

namespace {

using namespace mps;

constexpr size_t kScratchBytes = MPS_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

thread_local char g_err[256] = {0};

mps_status fail(mps_status st, const char* msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return st;
}

// Device address of this GPU's copy of `scratch` (looked up on first use).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

__global__ void k_fill_i32(int64_t n, int32_t* a, int32_t x) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) a[k] = x;
}
// Input types are FLUID/WALL/DUMMY/GHOST; anything else raises a status bit.
__global__ void k_check_type(int64_t n, const int8_t* t, int32_t* status) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n && (t[k] < MPS_FLUID || t[k] > MPS_GHOST)) atomicOr(status, ST_BADTYPE);
}
__global__ void k_iota_i32(int64_t n, int32_t* a) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) a[k] = (int32_t)k;
}
unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

// Bump allocation inside the scratch array, 256-byte aligned (base 0: a
// dry run that only counts the bytes).
struct Carve {
  uintptr_t base;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += ((size_t)count * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

}  // namespace

namespace mps {
const char* noctx_error() { return g_err[0] ? g_err : "no context"; }
}  // namespace mps

extern "C" mps_status mps_neighbors_noalloc(const mps_params* params, int64_t n,
                                            const double* pos, const int8_t* type,
                                            int32_t* cell_id, int32_t* count, int32_t* list,
                                            void* hip_stream) {
  g_err[0] = 0;
  if (check_params(params, n) != MPS_OK || !pos || !type)
    return fail(MPS_E_ARG, "invalid parameters or a NULL pointer");
  const mps_params& P = *params;
  const int dim = P.dim;
  const int ps = dim == 2 ? 2 : 4;
  const int kpad = (P.max_neigh + TEAM - 1) / TEAM * TEAM;
  const int64_t slots = ((n + SLICE - 1) / SLICE) * (int64_t)kpad * SLICE;
  const int ncell = P.grid_n[0] * P.grid_n[1] * (dim == 3 ? P.grid_n[2] : 1);
  const int64_t cells = scan_cells_padded(ncell);
  const int ntile = scan_tiles(ncell);

  // the layout: a dry run of the carving gives the bytes needed
  Carve dry{0};
  dry.take<double>(n * ps);      // positions in the kernels' layout, input order
  dry.take<double>(n * ps);      // sorted positions
  dry.take<int8_t>(n);           // types (ghosts marked), input order
  dry.take<int8_t>(n);           // types, sorted
  dry.take<int32_t>(n);          // ids, input order (identity)
  dry.take<int32_t>(n);          // ids, sorted
  for (int k = 0; k < 4; ++k) dry.take<int32_t>(n);  // cell, slot, perm, packed cell
  for (int k = 0; k < 3; ++k) dry.take<int32_t>(cells);  // counts, in-tile starts, starts
  dry.take<int32_t>(ntile);      // tile totals
  dry.take<int32_t>(n);          // list lengths
  dry.take<int32_t>(slots);      // lists (sliced layout)
  dry.take<int32_t>(1);          // status
  if (dry.used > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "mps_neighbors_noalloc needs %zu bytes of scratch for n = %lld, "
                  "max_neigh = %d, %d cells; the fixed array holds %zu",
                  dry.used, (long long)n, P.max_neigh, ncell, kScratchBytes);
    return fail(MPS_E_SCRATCH, msg);
  }

  void* base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return fail(MPS_E_DEVICE, hipGetErrorString(e));
  Carve cv{reinterpret_cast<uintptr_t>(base)};
  double* pos_in = cv.take<double>(n * ps);
  double* pos_s = cv.take<double>(n * ps);
  int8_t* type_c = cv.take<int8_t>(n);
  int8_t* type_s = cv.take<int8_t>(n);
  int32_t* id_in = cv.take<int32_t>(n);
  int32_t* id_s = cv.take<int32_t>(n);
  int32_t* cellid = cv.take<int32_t>(n);
  int32_t* slot = cv.take<int32_t>(n);
  int32_t* perm = cv.take<int32_t>(n);
  int32_t* pcell = cv.take<int32_t>(n);
  int32_t* cell_count = cv.take<int32_t>(cells);
  int32_t* cell_local = cv.take<int32_t>(cells);
  int32_t* cell_start = cv.take<int32_t>(cells);
  int32_t* tile_sum = cv.take<int32_t>(ntile);
  int32_t* nb_count = cv.take<int32_t>(n);
  int32_t* nb_list = cv.take<int32_t>(slots);
  int32_t* status = cv.take<int32_t>(1);

  hipStream_t s = (hipStream_t)hip_stream;
  // what must start at zero; the rest is written before it is read
  k_fill_i32<<<blocks256(cells), 256, 0, s>>>(cells, cell_count, 0);
  k_fill_i32<<<1, 256, 0, s>>>(1, status, 0);
  k_iota_i32<<<blocks256(n), 256, 0, s>>>(n, id_in);
  e = hipMemcpyAsync(type_c, type, (size_t)n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(MPS_E_DEVICE, hipGetErrorString(e));
  k_check_type<<<blocks256(n), 256, 0, s>>>(n, type_c, status);

  View v;
  std::memset(&v, 0, sizeof(v));
  v.n = n;
  v.kpad = kpad;
  v.max_neigh = P.max_neigh;
  v.nx = P.grid_n[0];
  v.ny = P.grid_n[1];
  v.nz = dim == 3 ? P.grid_n[2] : 1;
  v.ncell = ncell;
  for (int a = 0; a < 3; ++a) v.lo[a] = a < dim ? P.grid_lo[a] : 0.0;
  v.cs = P.cell_size;
  v.inv_cs = 1.0 / P.cell_size;
  v.re_lap = P.re_lap;
  v.re_lap2 = P.re_lap * P.re_lap;
  v.id = id_in;
  // the caller's [n][dim] positions into the kernels' vector layout (double2
  // in 2-D, padded double4 in 3-D), same order
  launch_gather_orig(v, pos, pos_in, dim, ps, s);
  // a1 on those positions; velocity, pressure and the two-phase fields are
  // absent (null), which the permutation skips
  v.pos = pos_in;
  v.pos_w = pos_s;
  v.type = type_c;
  v.type_w = type_s;
  v.id_w = id_s;
  v.cellid = cellid;
  v.slot = slot;
  v.cell_count = cell_count;
  v.cell_local = cell_local;
  v.tile_sum = tile_sum;
  v.ntile = ntile;
  v.cell_start = cell_start;
  v.perm = perm;
  v.pcell = pcell;
  v.nb_count = nb_count;
  v.nb_list = nb_list;
  v.status = status;
  launch_bin(v, dim, s);
  launch_permute(v, dim, MPS_FP64, s);
  // a2 and the export on the sorted arrays
  v.pos = pos_s;
  v.type = type_s;
  v.id = id_s;
  launch_neighbors(v, dim, MPS_FP64, s);
  launch_export_lists(v, cell_id, count, list, dim, s);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(MPS_E_DEVICE, hipGetErrorString(e));
  int32_t h = 0;
  e = hipMemcpyAsync(&h, status, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MPS_E_DEVICE, hipGetErrorString(e));
  if (h & ST_OVERFLOW) return fail(MPS_E_NEIGH_OVERFLOW, "more than max_neigh neighbours");
  if (h & ST_COINCIDENT) return fail(MPS_E_COINCIDENT, "two particles at distance 0");
  if (h & ST_NONFINITE) return fail(MPS_E_NONFINITE, "non-finite position");
  if (h & ST_BADTYPE) return fail(MPS_E_ARG, "invalid particle type");
  return MPS_OK;
}
