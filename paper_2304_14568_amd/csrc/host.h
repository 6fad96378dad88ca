// Host runtime declarations (context layout, packing, validation).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/admmbb.h"
#include "internal.h"

namespace admmbb {

admm_status validate_problem(const admm_problem* p, std::string* msg);
admm_status validate_options(const admm_options* o, std::string* msg);

// Host-side image of everything that goes to the device.
struct Packed {
  std::vector<Scen> scen;
  std::vector<int64_t> scen_nnz;  // nonzeros of each A_s as given (before chunk padding)
  std::vector<Pat> pat;
  std::vector<Tile> tiles;
  std::vector<Blk> blk, pblk;
  std::vector<uint32_t> rp;
  std::vector<uint16_t> col16;
  std::vector<int32_t> col32;
  std::vector<float> val;
  std::vector<uint16_t> val_lp;   // bf16 or fp16 bits
  std::vector<float> rscale;
  std::vector<float> rw, rpres;
  std::vector<double> rw64;       // c_s w_i per sorted row in fp64 (Gram matrices of the dense x-update)
  std::vector<int32_t> rorig;
  std::vector<float> b;           // A_s^T c_s W p per scenario (stacked)
  std::vector<double> b64;        // the same in fp64 (dense x-update right-hand sides)
  std::vector<float> dinv;        // Jacobi inverse diagonal (stacked), filled when requested
  std::vector<float> gdiag;       // (A_s^T c_s W A_s)_jj per scenario (stacked)
  std::vector<double> gdiag_mean; // per patient: mean over scenarios and spots of (A_s^T c_s W A_s)_jj
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
