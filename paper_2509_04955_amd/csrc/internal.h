// Internal declarations shared by the host planner, the C ABI and the HIP
// kernels of libqsim.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <mutex>
#include <string>
#include <new>
#include <stdexcept>
#include <vector>

#include "../../include/qsim.h"

namespace qs {

using cd = std::complex<double>;

// ------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

// Host work behind an ABI call: allocation failures and violated planner
// invariants become status codes instead of leaving through extern "C".
#define QS_ABI_TRY try {
#define QS_ABI_CATCH                                                         \
    }                                                                        \
    catch (const std::bad_alloc &) {                                         \
        qs::set_error("host allocation failed");                             \
        return QS_ENOMEM;                                                    \
    }                                                                        \
    catch (const std::exception &e) {                                        \
        qs::set_error("%s", e.what());                                       \
        return QS_EINVAL;                                                    \
    }
qs_status hip_fail(hipError_t e, const char *what);

#define QS_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return qs::hip_fail(e_, #call); \
    } while (0)

#define QS_CHECK(cond, code, ...)          \
    do {                                   \
        if (!(cond)) {                     \
            qs::set_error(__VA_ARGS__);    \
            return (code);                 \
        }                                  \
    } while (0)

// ------------------------------------------------------------- limits
constexpr int kMaxQubits = 40;
constexpr int kMaxTile = 14;          // tile qubits t (complex64: 2^14 * 8 B = 128 KiB LDS)
constexpr int kMaxTile128 = 13;       // complex128 tile limit (128 KiB)
constexpr int kMaxK = 6;              // widest fused block
constexpr int kMaxK128 = 5;
constexpr int kTileThreads = 256;     // threads per tile workgroup

// ------------------------------------------------------ device records
// One fused block as the tile kernel sees it.
// Block kinds: how the tile kernel applies a block's matrix.
enum : int32_t {
    BK_DENSE = 0,   // vector ALU, full 2^k x 2^k complex matrix
    BK_MFMA = 1,    // complex64, k = 4 or 5: MFMA with a pre-swizzled A operand
    BK_MONO = 2,    // monomial (one nonzero per column): y[dest(c)] = u_c x[c]
    BK_BDIAG = 3,   // permuted block-diagonal: classes of 2^sub rows/columns
    BK_PAULI = 4,   // Pauli rotation: y[k] = c psi[k] + d sigma(k^x) psi[k^x]
    BK_PAULIG = 5,  // k consecutive Pauli rotations with independent X parts, one lane per coset
    BK_SKIP = 6,    // folded into the preceding group (no work, no barrier)
    BK_BDMFMA = 7,  // complex64 permuted block-diagonal, classes of 2, 4 or 8, on MFMA (staged passes)
    BK_PERM = 8,    // k = 4 permutation (every nonzero entry 1): y[dest(c)] = x[c], no arithmetic
};

struct BlockDev {
    int32_t k;          // width
    int32_t kind;       // BK_*
    int32_t mat_off;    // offset (reals) of the matrix data in the plan's pool
    int32_t sub;        // BK_BDIAG: log2 of the class width, else 0
    int32_t pos[kMaxK]; // tile positions (ascending) of the block's qubits
    int32_t pad2[2];
};
static_assert(sizeof(BlockDev) == 48, "BlockDev layout");

// Launch arguments of one pass (passed by value).
struct PassArgs {
    int32_t t;          // tile qubits
    int32_t c;          // tile positions 0..c-1 are global qubits 0..c-1
    int32_t nblocks;
    int32_t block0;     // first block in the plan's block table
    int32_t hi[kMaxTile];   // global qubit of tile position c + j (ascending)
    int32_t apply_scale;    // multiply amplitudes by *scale on load
    int32_t want_norm;      // write FP64 sum |a|^2 partial per tile
    int32_t cl_off;         // block operands staged in LDS: pool elements
    int32_t cl_len;         //   [cl_off, cl_off + cl_len), 0 = none
};

// --------------------------------------------------------------- state
struct Prof;
}  // namespace qs

constexpr int kNumSlots = 8;
constexpr int kSlotTickets = 4;
struct qs_state_s {
    int n = 0;
    qs_dtype dtype = QS_C64;
    void *amp = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    // FP64 norm chain: slot[0] = norm of last pass, slot[1] = scale to apply next,
    // slots 2/3 scratch norm; slot kSlotTickets holds the tile-pass ticket
    // counter (64-bit, zero at creation) whose value the host mirrors in tickets.
    double *d_slots = nullptr;
    uint64_t tickets = 0;
    double *d_partials = nullptr;
    size_t partials_cap = 0;
    bool scale_pending = false;
};

namespace qs {

// Host gate after validation: full matrix with local bit j <-> q[j].
struct HGate {
    int kind = 0;
    int nq = 0;
    int q[8] = {0};
    double p[4] = {0, 0, 0, 0};
    std::vector<cd> m;   // 2^nq x 2^nq row-major
};

struct HBlock {
    std::vector<int> qubits;     // ascending
    std::vector<int64_t> members;
    std::vector<cd> U;           // 2^k x 2^k, local bit j <-> qubits[j] (empty for Pauli blocks)
    // Pauli-rotation block (a contracted window, see pauli.cpp): global X and
    // Z masks and the coefficients of y[k] = c psi[k] + d sigma(k^x) psi[k^x]
    bool pauli = false;
    uint64_t px = 0, pz = 0;
    cd pc, pd;
};

// A run of gates [begin, end) equal to one Pauli rotation (pauli.cpp).
struct PauliWindow {
    int64_t begin = 0, end = 0;
    uint64_t x = 0, z = 0;
    std::vector<int> support;    // ascending qubits the run touches
    cd c, d;
};

struct HPass {
    int t = 0, c = 0;
    std::vector<int> tile;       // ascending global qubits, size t
    int64_t block0 = 0, nblocks = 0;
};

}  // namespace qs

struct qs_plan_s {
    int n = 0;
    qs_contract_opts opts{};
    std::vector<qs::HGate> gates;
    std::vector<qs::HBlock> blocks;
    std::vector<qs::HPass> passes;
    // device copies (built on first use per dtype)
    int dev_ready[2] = {0, 0};
    qs::BlockDev *d_blocks[2] = {nullptr, nullptr};
    void *d_pool[2] = {nullptr, nullptr};
    std::vector<qs::BlockDev> h_blocks[2];
    std::vector<uint8_t> pass_wide[2];  // pass needs the wide kernel variant
    // pool range of the pass's block operands staged in LDS (len 0 = none)
    std::vector<int32_t> pass_cl_off[2], pass_cl_len[2];
    ~qs_plan_s();
};

namespace qs {

// ------------------------------------------------------------- host API
// gates.cpp
qs_status make_gate(const qs_gate &g, int n, HGate &out);
// planner.cpp
qs_status build_plan(qs_plan_s &p);
void block_matrix(const std::vector<HGate> &gates, HBlock &b);
// stage_lds: let passes stage their block operands in LDS (the single-state
// pass kernel); the batch kernel reads them from the pool.
qs_status plan_upload(qs_plan_s &p, qs_dtype dt, bool stage_lds = true);
// kernels_tile.hip: how the tile kernel will apply a block (BK_*); dest gets
// the monomial destinations when the block is monomial; lds: the pass stages
// its operands in LDS (dense complex64 k = 3 then also runs on MFMA)
int block_kind(const HBlock &b, int t, qs_dtype dt, std::vector<int> *dest, bool lds = false);
// log2 of the class width of a block's permuted block-diagonal form (BK_BDIAG)
int bdiag_log_width(const HBlock &b);
// whether the single-state pass kernel stages this pass's block operands in LDS
bool pass_staged(const std::vector<HBlock> &blocks, const HPass &ps, qs_dtype dt);
// packs blocks into passes and reorders them into execution order (in place)
void pack_passes(const qs_plan_s &p, std::vector<HBlock> &blocks, int t, int c,
                 std::vector<HPass> &out);
// solo (optional): units that always form a block of their own.  commute: a
// gate only follows the earlier gates it may not commute with (those acting
// non-diagonally on a qubit it shares, or any gate sharing a qubit it acts on
// non-diagonally); without it every gate follows all earlier gates sharing a
// qubit (Section 3.4's DAG)
void greedy_blocks(const std::vector<HGate> &gates, int n, int kmax, std::vector<HBlock> &blocks,
                   const std::vector<char> *solo = nullptr, bool commute = false);
// qubits on which a gate acts diagonally (its matrix has no entry between
// basis states that differ in that qubit); 0 for a gate without a matrix
uint64_t diagonal_qubits(const HGate &g);
// pauli.cpp: windows of Clifford gates around one diagonal one-qubit gate whose
// Clifford parts cancel (X weight at most max_x_weight); dense matrix of a
// Pauli block on its support
std::vector<PauliWindow> find_pauli_windows(const std::vector<HGate> &gates, int max_x_weight);
void pauli_block_matrix(HBlock &b);
// planner.cpp: the rotation windows the Pauli strategy contracts (X weight at
// most max_x_weight; diagonal rotations no wider than k_max are left to the
// greedy rule) and the blocks of that contraction: each window one rotation
// block (members: the window's gate range), every other gate merged greedily
// at k_max.  Members index `gates`; block matrices are not formed.
std::vector<PauliWindow> pauli_windows(const std::vector<HGate> &gates, int k_max, int max_x_weight);
void pauli_contract(const std::vector<HGate> &gates, int n, int k_max, const std::vector<PauliWindow> &win,
                    std::vector<HBlock> &blocks, bool commute = false);
int default_tile(qs_dtype dt);
// learned.cpp: features of one pass (kNumFeatures floats) and the learned
// per-window partition
constexpr int kNumFeatures = 17;
constexpr int kH1 = 64, kH2 = 64;
constexpr int kNumWeights = kH1 * kNumFeatures + kH1 + kH2 * kH1 + kH2 + kH2 + 1;
void pass_features(int n, qs_dtype dt, const HPass &ps, const std::vector<HBlock> &blocks, float *out);
qs_status learned_partition(qs_plan_s &p, int t, int c);
// mlp.hip: the active cost model
bool costmodel_loaded();
qs_status costmodel_predict_device(const float *features, int n_rows, float *out);

// ------------------------------------------------------- kernel launch
// kernels_plain.hip
struct Mat2 { double re[4], im[4]; };
qs_status launch_plain(qs_state_s &s, const HGate &g);
// kernels_smgp.hip: the gates in DAG layers with staggered multi-gate launches
qs_status launch_smgp(qs_state_s &s, const std::vector<HGate> &gates);
qs_status launch_scale(qs_state_s &s, const double *d_scale);
qs_status launch_set_basis(qs_state_s &s, uint64_t index);
qs_status launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st);
// kernels_tile.hip
// nparts (optional) receives the number of FP64 norm partials the pass wrote
qs_status launch_pass(qs_state_s &s, const qs_plan_s &p, const HPass &pass, int64_t pass_index, bool scale_in,
                      bool want_norm, uint64_t *nparts = nullptr);
qs_status launch_norm_reduce(qs_state_s &s, uint64_t nparts, double *d_out_slots);
qs_status launch_norm_full(qs_state_s &s, double *d_out_slots);
qs_status ensure_partials(qs_state_s &s, size_t count);
// kernels_expect.hip: Pauli-sum expectation, one read of the state per group
// of terms whose high X parts span at most kExpMaxD dimensions
constexpr int kExpMaxD = 9;            // span dimension of a group (coset = 2^D tiles)
constexpr int kExpMaxTerms = 9;        // terms per group (a random term adds one dimension)
constexpr int kExpCosetBits64 = 14;    // coset of 2^14 complex64 amplitudes = 128 KiB LDS
constexpr int kExpCosetBits128 = 13;   // 2^13 complex128 amplitudes = 128 KiB LDS
constexpr int kExpAmps64 = 16;         // amplitudes one thread stages per coset
constexpr int kExpAmps128 = 8;
constexpr size_t kExpTermsPerLaunch = 4096;   // user terms per launch (the API splits longer sums)
constexpr int kExpMaxAmps = 16;        // = max(kExpAmps64, kExpAmps128)
struct ExpectTerm {
    uint32_t zh;        // Z mask above the tile bits (the coset's sign)
    uint32_t xloc;      // X mask in coset coordinates (0: diagonal term)
    uint32_t zloc;      // Z mask in coset coordinates
    int32_t imag;       // pairs contribute Im(w) (|x&z| odd) instead of Re(w)
    double factor;      // +-2 for pairs (phase i^{|x&z|}), 1 for diagonal terms
    int32_t group;      // the term's group
    uint32_t x_off;     // xloc in LDS bytes
    // per staged index m of a thread (pairs: m < NA/2, diagonal: m < NA):
    uint32_t jm_off[kExpMaxAmps / 2];   // LDS byte offset of ins0(m T, h), h = top bit of xloc
    double sg[kExpMaxAmps];             // (-1)^parity(ins0(m T, h) & zloc), or of (m T) & zloc
};
static_assert(sizeof(ExpectTerm) == 192, "ExpectTerm layout");
struct ExpectGroup {
    uint32_t v[kExpMaxD];   // span basis over the high bits (at most 32), reduced echelon
    int32_t piv[kExpMaxD];  // pivot bit of each basis vector, ascending
    uint32_t mv[kExpMaxAmps];   // span vector of the tile coordinate of staged amplitude m
    int32_t term0, nterms;  // the group's terms (contiguous)
};
struct ExpectPlan {
    int n = 0, b = 0, l = 0, D = 0, threads = 0, log_cosets = 0;
    bool small = false;     // one-wave variant (state smaller than a full coset)
    uint64_t items = 0;
    uint32_t grid = 0;
    std::vector<ExpectTerm> terms;    // term 0 = identity (squared norm), then the caller's terms
    std::vector<ExpectGroup> groups;
};
// max_grid (0 = no limit) caps the workgroups of the launch
qs_status expect_plan(int n, qs_dtype dt, const uint64_t *x, const uint64_t *z, size_t n_terms, ExpectPlan &out,
                      uint32_t max_grid = 0);
size_t expect_scratch_bytes(const ExpectPlan &p);
// d_scratch: expect_scratch_bytes(p) device bytes, 256-byte aligned; *d_out
// receives the device address of the terms.size() results (term 0 = norm^2)
qs_status launch_expect(qs_state_s &s, const ExpectPlan &p, void *d_scratch, double **d_out);
// the library-held scratch of the no-allocation expectation (kernels_expect.hip):
// its device address on the current device, taken once per device; need
// beyond its size gives QS_ERANGE.  noalloc_lock serialises its users.
constexpr size_t kNoAllocMaxTerms = 2048;
constexpr uint32_t kNoAllocMaxGrid = 256;
qs_status noalloc_scratch(size_t need, void **ptr);
std::mutex &noalloc_lock();

// ------------------------------------------------------------ profiling
bool prof_on();
void prof_begin(hipStream_t st, int cls, double bytes, double flops);
void prof_end(hipStream_t st);

}  // namespace qs
