// Internal declarations shared by the host and device translation units of libspm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spm.h"

namespace spm {

constexpr int kMaxFun = 32;   // largest number of basis functions per cluster the kernels take
constexpr int kPieceEntries = 2048;   // largest piece of a block row in the S x dense product

int fail(int status, const std::string &msg);   // records msg, returns status

#define SPM_HIP(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::spm::fail(SPM_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

// Compute calls need the pattern's device tables (a planned pattern has host tables only).
#define SPM_NEED_DEVICE(p, name)                                                            \
    do {                                                                                    \
        if (!(p)->uploaded)                                                                 \
            return ::spm::fail(SPM_EINVAL, std::string(name) + ": pattern not uploaded");   \
    } while (0)

// Device copy of a host vector (owned by the pattern / tree handle).
template <typename T>
struct DevBuf {
    T *ptr = nullptr;
    size_t n = 0;
};

// Device copies of a tree's transform tables (two-scale matrices, input slots, level
// lists), uploaded on the first fast samplet transform and freed with the tree.  The
// tree is immutable, so the copies stay valid; the mutex guards the one upload.
struct TreeDevice {
    std::mutex mu;
    bool ready = false;
    double *q = nullptr;
    int32_t *nin = nullptr, *clist = nullptr;
    int64_t *qoff = nullptr, *sloff = nullptr, *slots = nullptr, *sob = nullptr, *perm = nullptr;
    std::vector<std::pair<int64_t, int64_t>> lvl;   // per level: offset and count in clist
    std::vector<int> lvl_mmax;                        // per level: largest number of inputs
    void release()
    {
        for (void *x : {(void *)q, (void *)nin, (void *)clist, (void *)qoff, (void *)sloff, (void *)slots,
                        (void *)sob, (void *)perm})
            if (x) (void)hipFree(x);
        q = nullptr; nin = clist = nullptr; qoff = sloff = slots = sob = perm = nullptr;
        ready = false;
    }
    ~TreeDevice() { release(); }
};

}  // namespace spm

struct spm_tree_s {
    int64_t n = 0;
    int32_t d = 0, leaf = 0, q = 0, m = 0;
    int32_t nc = 0, depth = 0;
    std::vector<double> pts;          // tree order, n x d
    std::vector<int64_t> perm;        // tree position -> original index
    std::vector<int64_t> pstart, psize;
    std::vector<int32_t> level, parent, son0, son1;
    std::vector<double> lo, hi;       // nc x d
    std::vector<int64_t> cstart;      // basis ranges, nc + 1
    // two-scale transforms
    std::vector<int32_t> nin, nscal;  // inputs and scaling functions handed up, per cluster
    std::vector<int64_t> qoff;        // offset of each cluster's Q (nin x nin, column-major)
    std::vector<double> qmat;
    std::vector<int64_t> slotoff;     // offset of each cluster's input slot list
    std::vector<int64_t> slots;       // input slots (tree-order point positions)
    std::unique_ptr<spm::TreeDevice> dev = std::make_unique<spm::TreeDevice>();
};

struct spm_pattern_s {
    int64_t n = 0, nnz = 0, n_stored = 0, n_tiles = 0;
    int32_t nc = 0;
    double macs = 0.0;
    bool masked = false;              // some tile positions are outside S
    int32_t max_rowlen = 0;           // longest block row (tiles)
    // host structure
    std::vector<int64_t> cstart;      // nc + 1
    std::vector<int32_t> nfun;        // nc
    std::vector<int64_t> blk_rp;      // nc + 1
    std::vector<int32_t> tile_row, tile_col, trans;   // n_tiles
    std::vector<int64_t> tile_off;    // n_tiles + 1
    std::vector<int64_t> diag_pos;    // stored positions of the diagonal entries (of the diagonal tiles), ascending
    std::vector<int64_t> colprefix;   // n_tiles: entries of the tile row before this tile
    std::vector<int64_t> rowbase, rowlen;  // nc: CSR position of the block row's first entry, entries per row
    std::vector<int32_t> diag_tile;   // nc
    // pieces of the block rows for the S x dense product: runs of tiles whose column
    // clusters are consecutive (a dense panel over a contiguous range of basis columns),
    // cut into pieces of whole 16-column chunks and at most kPieceEntries entries
    std::vector<int64_t> pc_rp;       // nc + 1
    std::vector<int64_t> pc_off, pc_g;   // element offset in the value array, first basis column
    std::vector<int32_t> pc_w;        // columns
    std::vector<int32_t> order;       // tile processing order (schedule)
    // grouped schedule of the FP64 product: groups of up to 4 consecutive clusters of
    // one size, and units = pairs of groups holding at least one output tile
    int32_t ng = 0, kmax = 4;         // groups, largest padded cluster size
    std::vector<int32_t> grp_mem;     // ng x 4 member clusters (-1 pads)
    std::vector<int32_t> grp_s, grp_g, grp_R;   // slot size, member count, rows (multiple of 16)
    std::vector<int64_t> gl_rp;       // ng + 1: union lists U(G) = union of the members' block rows
    std::vector<int32_t> gl_mu;       // cluster of each union entry
    std::vector<int32_t> gl_tile;     // entries x 4: tile (member k, mu) or -1
    std::vector<int32_t> unit_gr, unit_gc, unit_out;   // units; unit_out: units x 16 output tiles or -1
    std::vector<int32_t> unit_order;  // unit ids grouped by launch class, costly first
    std::vector<int64_t> pair_off;    // units + 1: offsets of each unit's middle-cluster list
    std::vector<int32_t> pair_a, pair_b;   // union-list entries of mu in U(G_r) and U(G_c)
    std::vector<int32_t> gl_nm;       // functions of the cluster of each union entry
    std::vector<int64_t> gl_offd;            // entries x 4: element offset of tile (member, mu), -1 absent
    std::vector<int64_t> stage_off;   // units + 1: stages of each unit
    std::vector<int32_t> stage_first; // first pair of each stage, relative to the unit's pair_off
    struct Launch {
        int32_t rb, cb, waves;
        int32_t smax_r, smax_c;   // largest slot of the row / column groups of the class
        int64_t first, count;
        int64_t out_tiles;        // output tiles of the class
        double exact_macs;        // sum over its output tiles (r, c) of n_r n_c sum_{mu in S_r cap S_c} n_mu
        double padded_macs;       // multiply-adds the kernels issue for it before block skipping
    };
    std::vector<Launch> launches;
    // tree levels of the clusters (optional, given at planning): with them the middle
    // clusters of a unit are ordered level by level and no stage mixes two levels, as the
    // split-precision product scales its operands per row and level
    std::vector<int32_t> clevel;      // nc, or empty
    int32_t nlev = 0;                 // 1 + largest level (0 without levels)
    std::vector<int32_t> gl_nml;      // entries: functions | level << 8 of the entry's cluster
    std::vector<int64_t> gl_offT;     // entries x 4: element offset of tile (mu, member), -1 absent
    // the middle clusters of each unit once more, ordered level by level, and stages of one
    // level each (the split-precision product; the FP64 and FP32 order is kept as it is)
    std::vector<int32_t> pair_a_lv, pair_b_lv;
    std::vector<int64_t> stage_off_lv;    // units + 1
    std::vector<int32_t> stage_first_lv;  // first pair of each stage (relative to the unit's pair_off)
    double padded_macs = 0.0;         // multiply-adds the grouped kernel issues (incl. padding)
    bool all_even = false;            // every cluster owns an even number of functions
    bool all_mult4 = false;           // every cluster owns a multiple of 4 functions
    // masked patterns only (entry-level upload)
    std::vector<int64_t> csr_rp;      // n + 1
    std::vector<int32_t> csr_col;
    std::vector<int64_t> csr_pos;     // n_stored: CSR position or -1
    // device copies: every table is carved from one block of device memory, owned by the
    // pattern (uploads that allocate) or by the caller (spm_pattern_upload_workspace)
    bool uploaded = false;
    void *dev_block = nullptr;
    bool owns_block = false;
    std::vector<double> tile_macs;    // n_tiles: exact multiply-adds of each output tile (planning only)
    spm::DevBuf<int64_t> d_cstart, d_blk_rp, d_tile_off, d_colprefix, d_rowbase, d_rowlen, d_csr_pos;
    spm::DevBuf<int64_t> d_pc_rp, d_pc_off, d_pc_g;
    spm::DevBuf<int32_t> d_pc_w;
    spm::DevBuf<int32_t> d_nfun, d_tile_row, d_tile_col, d_trans, d_diag_tile, d_order;
    spm::DevBuf<int32_t> d_grp_mem, d_grp_s, d_grp_g, d_grp_R, d_gl_mu, d_gl_tile, d_unit_gr, d_unit_gc, d_unit_out,
        d_unit_order;
    spm::DevBuf<int64_t> d_gl_rp, d_pair_off, d_gl_offd, d_stage_off;
    spm::DevBuf<int32_t> d_pair_a, d_pair_b, d_gl_nm, d_stage_first;
    spm::DevBuf<int32_t> d_clevel, d_gl_nml, d_stage_first_lv, d_pair_a_lv, d_pair_b_lv;
    spm::DevBuf<int64_t> d_gl_offT, d_stage_off_lv;
    spm::DevBuf<uint8_t> d_keep;      // n_stored, masked patterns only
    spm::DevBuf<int64_t> d_diag_pos;
    spm::DevBuf<double> d_partial;    // reduction partials
};

namespace spm {
size_t pattern_device_bytes(const spm_pattern_s *p);
// copies the tables into ws (bytes >= pattern_device_bytes), or into a block it
// allocates when ws is null
int upload_pattern_device(spm_pattern_s *p, void *ws, size_t bytes, hipStream_t s);
void free_pattern_device(spm_pattern_s *p);
}  // namespace spm

namespace spm {
int launch_gemm(spm_pattern_s *p, int prec, const void *A, int ta, const void *B, int tb, void *C, hipStream_t s);
size_t gemm_ws_bytes(spm_pattern_s *p, int prec, int ta, int tb);
int gemm_ws(spm_pattern_s *p, int prec, const void *A, int ta, const void *B, int tb, void *C, void *ws, hipStream_t s);
size_t ws_align(size_t x);
int launch_reduce(spm_pattern_s *p, int op, int prec, const void *x, const void *y, const double *vec, double alpha,
                  int post, double scale, double *out, hipStream_t s);
int launch_axpy(spm_pattern_s *p, int prec, double alpha, const void *X, double beta, void *Y, hipStream_t s);
int launch_convert(spm_pattern_s *p, int pf, const void *X, int pt, void *Y, hipStream_t s);
}  // namespace spm
