// Host runtime declarations (context layout, packing, validation).
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/admmbb.h"
#include "internal.h"

namespace admmbb {

// Host memory of the packed arrays: page-locked (hipHostMalloc) while a
// packing has pinned budget left and the block is large, so that its upload
// runs at the link's DMA rate; otherwise (or when no device is there) the
// ordinary heap.  host_free releases either kind.
void* host_alloc(size_t bytes);
void host_free(void* p) noexcept;
// Pinned budget of the packing on this thread (bytes; 0 = none), restored on
// scope exit.
struct PinnedBudget {
  explicit PinnedBudget(size_t bytes);
  ~PinnedBudget();
  size_t saved;
};

// Allocator whose value-less construct leaves elements uninitialised: for the
// large packed arrays, every element of which the (parallel) packing writes,
// so that growing them costs no single-threaded zero fill.  Storage from
// host_alloc.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) {}
  T* allocate(size_t n) { return static_cast<T*>(host_alloc(n * sizeof(T))); }
  void deallocate(T* p, size_t) noexcept { host_free(p); }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    if constexpr (sizeof...(Args) == 0)
      ::new (static_cast<void*>(p)) U;
    else
      ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <class T, class U>
bool operator==(const NoInit<T>&, const NoInit<U>&) {
  return true;
}
template <class T, class U>
bool operator!=(const NoInit<T>&, const NoInit<U>&) {
  return false;
}
template <class T>
using RawVec = std::vector<T, NoInit<T>>;

admm_status validate_problem(const admm_problem* p, std::string* msg);
admm_status validate_options(const admm_options* o, std::string* msg);

// Host-side image of everything that goes to the device.
struct Packed {
  std::vector<Scen> scen;
  std::vector<int64_t> scen_nnz;  // nonzeros of each A_s as given (before chunk padding)
  std::vector<Pat> pat;
  std::vector<Tile> tiles;
  std::vector<Blk> blk, pblk;
  RawVec<uint32_t> rp;
  RawVec<uint16_t> col16;
  RawVec<int32_t> col32;
  RawVec<float> val;
  RawVec<uint16_t> val_lp;        // bf16 or fp16 bits
  RawVec<float> rscale;
  RawVec<float> rw, rpres;
  RawVec<double> rw64;            // c_s w_i per sorted row in fp64 (Gram matrices of the dense x-update)
  RawVec<int32_t> rorig;
  // sliced layout (MatDev FMT_SELL), one array per (patient, scenario) in
  // scenario order, uploaded at sell_base of each; slice offsets of all
  // scenarios in soff (one terminal entry after each scenario's slices)
  std::vector<RawVec<float>> sell_val;
  std::vector<RawVec<uint16_t>> sell_col16;
  std::vector<RawVec<uint16_t>> sell_val_lp;
  std::vector<uint32_t> soff;
  int64_t sell_total = 0;         // chunk slots of the sliced layout over all scenarios
  std::vector<float> b;           // A_s^T c_s W p per scenario (stacked)
  std::vector<double> b64;        // the same in fp64 (dense x-update right-hand sides)
  std::vector<float> dinv;        // Jacobi inverse diagonal (stacked), filled when requested
  std::vector<float> gdiag;       // (A_s^T c_s W A_s)_jj per scenario (stacked)
  std::vector<double> gdiag_mean; // per patient: mean over scenarios and spots of (A_s^T c_s W A_s)_jj
  std::vector<double> gdiag_max;  // per scenario: max_j (A_s^T c_s W A_s)_jj in fp64
  std::vector<std::vector<double>> g0;  // per patient: 2 sum_s b_s
  std::vector<float> lb, ub;      // per patient stacked
  int64_t vec_total = 0, zvec_total = 0, part_total = 0, nnz_total = 0, rows_total = 0;
  int nmax = 0, mmax = 0;
  bool col16_used = true;
};

admm_status pack_problems(const admm_problem* probs, int num_patients, const admm_options& o, Packed* out,
                          std::string* msg);

// bf16 / fp16 bit patterns with round-to-nearest-even
uint16_t to_bf16_bits(float v);
uint16_t to_f16_bits(float v);

}  // namespace admmbb
