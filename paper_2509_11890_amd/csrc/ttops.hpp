// Memory-bound helper kernels (permutations, core builders, vector updates, dots).
#pragma once

#include <vector>

#include "common.hpp"

namespace ttipm {

// Independent permutations (as permute, alpha = 1), up to 16 per launch.
struct PermJob {
  const double* in;
  double* out;
  std::vector<long> dims;
  std::vector<int> perm;
};
void permute_many(const std::vector<PermJob>& jobs, hipStream_t s);
// out = alpha * permute(in): input row-major with dims; output dims are dims[perm[0]], dims[perm[1]], ...
void permute(const double* in, double* out, const std::vector<long>& dims, const std::vector<int>& perm,
             hipStream_t s, double alpha = 1.0);
// Place src [n0][mid][n1] into dst [N0][mid][N1] at (o0, o1), scaled by alpha (other entries untouched).
void place_block(const double* src, int n0, long mid, int n1, double* dst, int N0, int N1, int o0, int o1,
                 double alpha, hipStream_t s);
// Per-core Kronecker product of TT-matrix cores A [ra][ma][na][sa] and B [rb][mb][nb][sb].
void kron_core(const double* A, int ra, int ma, int na, int sa, const double* B, int rb, int mb, int nb, int sb,
               double* C, hipStream_t s);
// diag_TT core from a TT-vector core v [r][m][s] -> D [r][m][m][s].
void diag_core(const double* v, int r, int m, int s, double* D, hipStream_t st);
// TT matvec core: y [(R r)][mo][(S s)] from A [R][mo][mi][S] and x [r][mi][s].
void matvec_core(const double* A, int R, int mo, int mi, int S, const double* x, int r, int s, double* y,
                 hipStream_t st);
// TT matmat core: C [(R r)][mo][nk][(S s)] from A [R][mo][mi][S] and B [r][mi][nk][s].
void matmat_core(const double* A, int R, int mo, int mi, int S, const double* B, int r, int nk, int s, double* C,
                 hipStream_t st);
// Strided 2D block copy: dst[i*dst_ld + j] = src[i*src_ld + j].
void copy2d(const double* src, long src_ld, double* dst, long dst_ld, int rows, int cols, hipStream_t s);
// y = a x + b y
void axpby(long n, double a, const double* x, double b, double* y, hipStream_t s);
void fill(long n, double v, double* y, hipStream_t s);
// y += sign * sum_j coef[j] V_j  (coef on device)
void gemv_update(long n, int k, const double* V, long ld, const double* coef, double sign, double* y,
                 hipStream_t s);
// out[j] = <V_j, w>, j < k (deterministic).  part needs mdot_part_size(k) doubles.
void mdot(long n, int k, const double* V, long ld, const double* w, double* out, double* part, hipStream_t s);
size_t mdot_part_size(int k);

}  // namespace ttipm
