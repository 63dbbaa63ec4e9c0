// Host-side hierarchical partition and box schedule (Sec. 3; Algorithm 1 order).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace rsrs {

struct Tree {
  int dim = 2, qbits = 20, leaf_size = 64, nlevels = 0;
  int64_t n = 0;
  // per box (ids sorted by (level, Morton code))
  std::vector<int32_t> level;
  std::vector<int32_t> coords;     // nbox x dim
  std::vector<int64_t> parent;
  std::vector<uint8_t> is_leaf;
  std::vector<int64_t> pt_begin, pt_end;
  std::vector<int64_t> child_off, child_ids;   // CSR of children (ascending ids)
  std::vector<int64_t> perm;       // tree position -> user index
  // per level l (index l): boxes at level l, and neighbour CSR for them
  std::vector<std::vector<int64_t>> level_boxes;
  std::vector<std::vector<int64_t>> nb_off, nb_ids;
  int64_t nbox() const { return (int64_t)level.size(); }
  int64_t npts(int64_t b) const { return pt_end[b] - pt_begin[b]; }
};

// Box order and active counts for rank k.
struct Schedule {
  int k = 0;
  std::vector<int32_t> colour;     // -1 when not processed
  std::vector<int64_t> b_count, l_count;
  int64_t root_count = 0;
  // levels nlevels..1, each a list of colour classes (box ids ascending)
  std::vector<int> levels;
  std::vector<std::vector<std::vector<int64_t>>> classes;
};

// Returns empty string on success, else an error message.
std::string build_tree(const double* pts, int64_t n, int dim, int leaf_size, int qbits,
                       const double* lo, double side, Tree& t);
void make_schedule(const Tree& t, int k, Schedule& s);
int64_t samples_required(const Tree& t, const Schedule& s, int k, int p);
// Algorithmic flops, bytes and stored entries of a fixed-rank factorization;
// subset_p >= 0: boxes read s_B = min(s, l + k + subset_p) sample columns.
void work_model(const Tree& t, const Schedule& s, int k, int64_t nsamples, bool sym, int esize,
                int subset_p, double* flops, double* bytes, int64_t* stored);

}  // namespace rsrs
