// Partitioned low-rank (PLR) powers, §5: record layout shared by the host
// planner and the kernels, work descriptors and launchers.
#pragma once

#include "ssm_internal.h"

namespace ssmc {

constexpr int kPlrLeaf = 16;       // dense diagonal leaves are 16 x 16
constexpr int kPlrRC = 32;         // largest rank kept per off-diagonal block
constexpr int kPlrMaxS = 128;      // largest off-diagonal block (padded m 256)
constexpr int kPlrRankSlots = 32;  // rank-table entries per record (2 (2^D - 1) <= 30)

// levels D of the dyadic partition down to 16 x 16 leaves
__host__ __device__ constexpr int plr_levels(int mp) {
  return mp == 256 ? 4 : mp == 128 ? 3 : mp == 64 ? 2 : mp == 32 ? 1 : 0;
}
// elements of one record: per level 2^d blocks of 2 s kPlrRC, then the leaves
__host__ __device__ constexpr int64_t plr_rec_elems(int mp) {
  return (int64_t)plr_levels(mp) * 2 * mp * kPlrRC + (int64_t)mp * kPlrLeaf;
}
// U' of block (d, g, side) within a record (V^T follows at + s kPlrRC)
__host__ __device__ constexpr int64_t plr_block_off(int mp, int d, int g, int side) {
  return (int64_t)(d - 1) * 2 * mp * kPlrRC + (int64_t)(2 * g + side) * 2 * (mp >> d) * kPlrRC;
}
__host__ __device__ constexpr int64_t plr_leaf_off(int mp) { return (int64_t)plr_levels(mp) * 2 * mp * kPlrRC; }
__host__ __device__ constexpr int plr_rank_index(int d, int g, int side) {
  return ((1 << (d - 1)) - 1) * 2 + 2 * g + side;
}

// One compression workgroup: the off-diagonal block (d, g, side) of P_k of
// operator op, or (d == 0) the copy of its dense leaves.
struct PlrJob {
  int32_t op, k, d, g, side, reserved[3];
};

struct PlrCompressParams {
  const OpDev* ops;
  const PlrJob* jobs;
  const double* pw;        // FP64 powers (OpDev::pw offsets)
  void* rec;               // records, compute type
  const int64_t* rec_off;  // per operator: element offset of its stage-0 record
  int32_t* ranks;          // rank table
  const int32_t* rank_off; // per operator: first entry of its stage-0 record
  double* qs;              // FP64 scratch, kPlrRC kPlrMaxS per job
  double tol2;             // squared Frobenius tolerance per block
};

// Rows [row0, row0 + plr_unit_rows) of sequence seq (4 waves of NT 16-row blocks).
struct PlrUnit {
  int32_t seq, row0;
};

struct PlrStageParams {
  const SeqDev* seqs;
  const PlrUnit* units;
  int32_t n_units;
  int32_t k;
  const void* rec;
  const int64_t* rec_off;
  const int32_t* ranks;
  const int32_t* rank_off;
  const void* xin;
  void* xout;
};

// rows of one PLR stage workgroup
constexpr int plr_unit_rows(int compute) { return compute == DT_F64 ? 64 : 128; }

size_t plr_compress_lds(int max_s);
hipError_t launch_plr_compress(int compute, const PlrCompressParams& prm, int n_jobs, int max_s,
                               hipStream_t st);
hipError_t launch_stage_plr(int mp, int compute, const PlrStageParams& prm, hipStream_t st);

}  // namespace ssmc
