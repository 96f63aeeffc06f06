// C ABI of libhp2sph: plans, workspace, stage sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <unordered_set>
#include <vector>

#include "../../include/hp2sph.h"
#include "kernels.h"
#include "tables.h"

namespace hp2sph {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Device copy of one nside's tables in precision T.
template <class T>
struct DevTables {
    std::vector<std::unique_ptr<DevBuf>> owned;
    T* ana[4] = {};
    T* givens[4] = {};
    FftTab<T> fft{};

    T* upload(const std::vector<double>& v) {
        std::vector<T> tmp(v.begin(), v.end());
        auto b = std::make_unique<DevBuf>();
        b->bytes = std::max<size_t>(tmp.size(), 1) * sizeof(T);
        if (hipMalloc(&b->p, b->bytes) != hipSuccess) throw std::bad_alloc();
        if (!tmp.empty() && hipMemcpy(b->p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            throw std::runtime_error("hipMemcpy failed");
        T* out = static_cast<T*>(b->p);
        owned.push_back(std::move(b));
        return out;
    }
};

template <class I>
I* upload_int(std::vector<std::unique_ptr<DevBuf>>& owned, const std::vector<I>& v) {
    auto b = std::make_unique<DevBuf>();
    b->bytes = std::max<size_t>(v.size(), 1) * sizeof(I);
    if (hipMalloc(&b->p, b->bytes) != hipSuccess) throw std::bad_alloc();
    if (!v.empty() && hipMemcpy(b->p, v.data(), v.size() * sizeof(I), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed");
    I* out = static_cast<I*>(b->p);
    owned.push_back(std::move(b));
    return out;
}

// Workgroup -> (problem, tile) maps of one grouped GEMM, one per candidate
// schedule (HP2SPH_SCHED_*), and the one the launches use.
struct GemmSched {
    int32_t* tmap = nullptr;      // active map
    int slots = 0;                // its length (workgroups per launch)
    int sched = HP2SPH_SCHED_XCD_ROUND_ROBIN;
    int32_t* maps[HP2SPH_NSCHED] = {};
    int nslots[HP2SPH_NSCHED] = {};
    void use(int c) {
        sched = c;
        tmap = maps[c];
        slots = nslots[c];
    }
};

template <class T>
struct GemmList : GemmSched {
    GemmProblem<T>* dev = nullptr;
    int n = 0, tiles = 0;
    std::vector<GemmProblem<T>> host;   // the uploaded list (launch order)
};

struct Group {
    int nside = 0;
    int index = 0;                    // position in the plan's group list
    std::vector<int> members;         // batch indices
    GroupDims dims{};
    double pole_w[3] = {0, 0, 0};
    std::vector<std::unique_ptr<DevBuf>> owned;
    RingTab rings{};
    DevTables<double> t64;
    DevTables<float> t32;
    double* syn[4] = {};              // synthesis matrices (FP64)
    double* synT[4] = {};             // their transposes [h][l'] (equal-weight analysis, staged)
    int64_t* d_map_off = nullptr;     // per member: offset of its map (doubles)
    int64_t* d_alm_off = nullptr;     // per member: offset of its alm (complex)
    int64_t* d_cl_off = nullptr;
    int32_t* d_lmax = nullptr;
    int32_t* d_pack_tiles = nullptr;   // (m, l0) of the pack tiles
    int n_pack_tiles = 0;
    int lmax_max = 0;
    // workspace regions (byte offsets from the plan's workspace; each group
    // has its own, so that one launch can serve every group): D, U and, by
    // mode, the refinement's Df (FP64 ring coefficients), Dr (FP32 residual
    // coefficients), Ua (FP32 a0) or the equal-weight analysis' Ua (FP64 a),
    // Wf and Wr (longitude sums of the maps and of the residual)
    size_t off_D = 0, off_U = 0;
    size_t off_Df = 0, off_Dr = 0, off_Ua = 0, off_Wf = 0, off_Wr = 0;
    size_t bytes_D = 0, bytes_U = 0;
    int64_t rows_D[4] = {}, rows_U[4] = {};
    size_t blk_off_D[4] = {}, blk_off_U[4] = {};   // byte offset of each block in its region
    // strategy: per-order tables (fused colatitude fit + Givens sweeps) or staged
    bool tables = false;
    // device GEMM problem lists
    GemmList<double> ana64, syn64, syn64_staged;
    GemmList<float> ana32;       // FP32 analysis of FP32 Dsym (second pass of the refinement)
    GemmList<float> ana32_b64;   // FP32 analysis reading FP64 Dsym (single FP32 pass, first pass of the refinement)
    GemmList<double> adj64;      // equal-weight analysis: transposed evaluation (adjoint of the synthesis GEMM)
};

template <class T>
const GemmList<T>& gemm_list(const Group& G);
template <>
const GemmList<double>& gemm_list<double>(const Group& G) { return G.ana64; }
template <>
const GemmList<float>& gemm_list<float>(const Group& G) { return G.ana32_b64; }

}  // namespace
}  // namespace hp2sph

namespace hp2sph {
namespace {
// HIP-event timing of stage launches (see hp2sph_profile in hp2sph.h)
struct Profiler {
    bool on = false;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[HP2SPH_NSTAGES] = {};
    int launches[HP2SPH_NSTAGES] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipError_t drain() {
        for (auto& r : pending) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e != hipSuccess) return e;
            float t = 0.f;
            e = hipEventElapsedTime(&t, r.a, r.b);
            if (e != hipSuccess) return e;
            ms[r.stage] += t;
            launches[r.stage] += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
        return hipSuccess;
    }
    ~Profiler() {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
thread_local Profiler* g_prof = nullptr;   // profiler of the plan being executed
}  // namespace
}  // namespace hp2sph

struct hp2sph_plan_s {
    hp2sph::Profiler prof;
    int batch = 0;
    int mode = 0;
    int device = 0;
    std::vector<int32_t> nside, lmax;
    std::vector<int64_t> map_off, alm_off, cl_off;
    int64_t total_pix = 0, total_alm = 0, total_cl = 0;
    std::vector<std::unique_ptr<hp2sph::Group>> groups;   // descending nside
    size_t ws_bytes = 0;
    int strategy = 0;                 // requested HP2SPH_STRATEGY_*
    // work-list launches: one descriptor per group (device and host copies),
    // the spans of groups that share the ring kernels' thread count, and the
    // persistent grid of the fold (0: one workgroup per item)
    std::vector<std::unique_ptr<hp2sph::DevBuf>> owned;
    std::vector<hp2sph::GroupDesc> gdesc;
    hp2sph::GroupDesc* d_gdesc = nullptr;
    std::vector<std::pair<int, int>> ring_spans;
    int fold_grid = 0;
    int pack_maps = 32;               // maps per pack tile (mode-major layout): 16, 32 or 64
    int ring_order = 0;               // item order of the ring transform: 0 (XCD-aware), 1, 2
    int ring_threads = 256;           // threads of the ring transform up to nside 1024: 256 or 512
    // per-map offsets of the whole batch (C_l in one launch)
    int64_t* d_alm_off = nullptr;
    int64_t* d_cl_off = nullptr;
    int32_t* d_lmax = nullptr;
    int lmax_max = 0;
    // the analysis GEMMs of every group merged into one list per role (B and
    // C offsets from the workspace base): FP64 analysis; FP32 analysis of
    // FP64 ring coefficients; FP64 synthesis; FP32 analysis of FP32 ones
    hp2sph::GemmList<double> m_ana64, m_syn64;
    hp2sph::GemmList<float> m_ana32_b64, m_ana32;
};

using namespace hp2sph;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultJacobi = 3;   // the iteration count HEALPix uses by default (Sec. 2.2)
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <class T>
void fill_fft(DevTables<T>& d, const HostTables& h, std::vector<std::unique_ptr<DevBuf>>& owned) {
    d.fft.twiddle = d.upload(h.twiddle);
    d.fft.roots = d.upload(h.roots);
    d.fft.chirp = d.upload(h.chirp);
    d.fft.chirpfft = d.upload(h.chirpfft);
    d.fft.rootoff = upload_int(owned, h.rootoff);
    d.fft.chirpoff = upload_int(owned, h.chirpoff);
    d.fft.chirpfftoff = upload_int(owned, h.chirpfftoff);
    d.fft.chirpm = upload_int(owned, h.chirpm);
    d.fft.fft_max = h.fft_max;
}

// Givens tables padded in t to a multiple of the sweep pass length
std::vector<double> pad_givens(const std::vector<double>& g, int nl, int T, int tpad) {
    std::vector<double> out(size_t(nl) * tpad * 2, 0.0);
    for (int lp = 0; lp < nl; ++lp)
        for (int t = 0; t < T; ++t) {
            out[(size_t(lp) * tpad + t) * 2] = g[(size_t(lp) * T + t) * 2];
            out[(size_t(lp) * tpad + t) * 2 + 1] = g[(size_t(lp) * T + t) * 2 + 1];
        }
    return out;
}

// Column order of Dsym / U (see GroupDims): map-major for the staged
// strategy, mode-major for the per-order tables.
void set_layout(GroupDims& d, bool modemajor) {
    d.modemajor = modemajor ? 1 : 0;
    for (int kp = 0; kp < 2; ++kp) {
        d.cm[kp] = modemajor ? 2 : d.Npm[kp];
        d.ck[kp] = modemajor ? 2 * int64_t(d.nmaps) : 2;
    }
}

// Shapes of a group's blocks and workspace rows (host arithmetic only).
void init_dims(Group& G) {
    GroupDims& d = G.dims;
    d.nside = G.nside;
    d.p = 2 * G.nside;
    d.nmaps = int(G.members.size());
    for (int b = 0; b < 4; ++b) {
        BlockShape bs = block_shape(G.nside, b);
        d.nl[b] = bs.nl;
        d.nk[b] = bs.nk;
        d.lmin[b] = bs.lmin;
        const int T = std::max(bs.nsweep, 1);
        d.tpad[b] = (T + 7) / 8 * 8;
    }
    d.Npm[0] = 2 * d.nk[0];
    d.Npm[1] = 2 * d.nk[2];
    d.N[0] = int64_t(d.nmaps) * d.Npm[0];
    d.N[1] = int64_t(d.nmaps) * d.Npm[1];
    set_layout(d, false);
    // workspace sizes (FP64 elements; FP32 stages alias the same bytes)
    const int K = 2 * G.nside + 1;
    G.bytes_D = 0;
    G.bytes_U = 0;
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        G.rows_D[b] = K;
        G.rows_U[b] = d.nl[b];
        G.blk_off_D[b] = G.bytes_D;
        G.blk_off_U[b] = G.bytes_U;
        G.bytes_D += align_up(size_t(K) * d.N[kpar] * sizeof(double));
        G.bytes_U += align_up(size_t(d.nl[b]) * d.N[kpar] * sizeof(double));
    }
}

void build_group(hp2sph_plan_t plan, Group& G) {
    HostTables h;
    build_tables(G.nside, h, true);
    const int p = h.p;
    GroupDims& d = G.dims;
    init_dims(G);
    for (int i = 0; i < 3; ++i) G.pole_w[i] = h.pole_w[i];

    // rings
    std::vector<int64_t> st;
    std::vector<int32_t> nn;
    std::vector<int8_t> sh;
    for (auto& r : h.rings) {
        st.push_back(r.start);
        nn.push_back(int32_t(r.n));
        sh.push_back(r.phi0 != 0.0 ? 1 : 0);
    }
    G.rings.start = upload_int(G.owned, st);
    G.rings.n = upload_int(G.owned, nn);
    G.rings.shifted = upload_int(G.owned, sh);

    const bool need64 = true;   // FP64 tables: analysis in F64 mode, always for synthesis
    const bool need32 = (plan->mode == HP2SPH_F32_REFINE || plan->mode == HP2SPH_F32);
    for (int b = 0; b < 4; ++b) {
        const int T = std::max(block_shape(G.nside, b).nsweep, 1);
        std::vector<double> gp = pad_givens(h.givens[b], d.nl[b], T, d.tpad[b]);
        if (need64) {
            G.t64.ana[b] = G.t64.upload(h.ana[b]);
            G.t64.givens[b] = G.t64.upload(gp);
        }
        if (need32) {
            G.t32.ana[b] = G.t32.upload(h.ana[b]);
            G.t32.givens[b] = G.t32.upload(gp);
        }
        G.syn[b] = G.t64.upload(h.syn[b]);
        if (plan->mode == HP2SPH_EQUAL_WEIGHT) {
            // [l'][h] (2 nside + 1 columns) -> [h][l']
            const int K = 2 * G.nside + 1, nl = d.nl[b];
            std::vector<double> t(size_t(K) * nl);
            for (int lp = 0; lp < nl; ++lp)
                for (int hh = 0; hh < K; ++hh) t[size_t(hh) * nl + lp] = h.syn[b][size_t(lp) * K + hh];
            G.synT[b] = G.t64.upload(t);
        }
    }
    fill_fft(G.t64, h, G.owned);

    // per-member offsets
    std::vector<int64_t> mo, ao, co;
    std::vector<int32_t> lm;
    G.lmax_max = 0;
    for (int i : G.members) {
        mo.push_back(plan->map_off[i]);
        ao.push_back(plan->alm_off[i]);
        co.push_back(plan->cl_off[i]);
        lm.push_back(plan->lmax[i]);
        G.lmax_max = std::max(G.lmax_max, int(plan->lmax[i]));
    }
    G.d_map_off = upload_int(G.owned, mo);
    G.d_alm_off = upload_int(G.owned, ao);
    G.d_cl_off = upload_int(G.owned, co);
    G.d_lmax = upload_int(G.owned, lm);
    {
        std::vector<int32_t> pt = pack_tiles(p);
        G.n_pack_tiles = int(pt.size() / 2);
        G.d_pack_tiles = upload_int(G.owned, pt);
    }

}

template <class T>
Blocks4<T> blocks_at(void* ws, size_t off, const Group& G, const int64_t* rows) {
    Blocks4<T> out;
    char* base = static_cast<char*>(ws) + off;
    size_t o = 0;
    for (int b = 0; b < 4; ++b) {
        out.p[b] = reinterpret_cast<T*>(base + o);
        o += align_up(size_t(rows[b]) * G.dims.N[b >> 1] * sizeof(double));
    }
    return out;
}

template <class T>
Blocks4<const T> cblocks(Blocks4<T> b) {
    Blocks4<const T> o;
    for (int i = 0; i < 4; ++i) o.p[i] = b.p[i];
    return o;
}

// ---------------------------------------------------------------------------
// GEMM problem lists and the per-order tables
// ---------------------------------------------------------------------------

// Smallest half-ring row that carries mode m in the analysis: polar ring j
// holds modes |k| <= 2j only, so rows h < m/2 are zero for mode m (and the
// pole row carries m = 0 only).
int first_row(int m) { return m == 0 ? 0 : (m + 1) / 2; }

// The alternatives to xcd_tile_map (HP2SPH_SCHED_XCD_ROUND_ROBIN) for a
// finalized problem list in launch order (longest first):
//   XCD_BALANCED: each problem to the XCD with the least work so far (tiles
//     times K, longest-processing-time-first), its tiles kept together;
//     workgroup w runs on XCD w mod 8 (the hardware deals workgroups to the 8
//     XCDs in turn), entries of -1 pad the XCDs to equal length;
//   LINEAR: workgroup w runs tile w of the list (no XCD placement);
//   LINEAR_ROWS: problems in list order, and within a problem the row tiles
//     of each column panel consecutively (tile = row * tiles_n + col, row
//     fastest).
template <class T>
std::vector<int32_t> schedule_map(const std::vector<GemmProblem<T>>& v, int total_tiles, int sched) {
    constexpr int kXcd = 8;
    const int n = int(v.size());
    auto tiles_of = [&](int i) { return (i + 1 < n ? v[i + 1].tile_begin : total_tiles) - v[i].tile_begin; };
    std::vector<int32_t> out;
    if (sched == HP2SPH_SCHED_LINEAR) {
        for (int i = 0; i < n; ++i)
            for (int t = 0; t < tiles_of(i); ++t) {
                out.push_back(i);
                out.push_back(t);
            }
        return out;
    }
    if (sched == HP2SPH_SCHED_LINEAR_ROWS) {
        for (int i = 0; i < n; ++i) {
            const int tn = v[i].tiles_n, tm = tiles_of(i) / tn;
            for (int c = 0; c < tn; ++c)
                for (int r = 0; r < tm; ++r) {
                    out.push_back(i);
                    out.push_back(r * tn + c);
                }
        }
        return out;
    }
    std::vector<std::vector<int32_t>> per(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    for (int i = 0; i < n; ++i) {
        const int x = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += int64_t(tiles_of(i)) * v[i].K;
        for (int t = 0; t < tiles_of(i); ++t) {
            per[x].push_back(i);
            per[x].push_back(t);
        }
    }
    size_t len = 0;
    for (auto& p : per) len = std::max(len, p.size() / 2);
    out.assign(2 * len * kXcd, -1);
    for (int x = 0; x < kXcd; ++x)
        for (size_t j = 0; j < per[x].size() / 2; ++j) {
            out[2 * (j * kXcd + x)] = per[x][2 * j];
            out[2 * (j * kXcd + x) + 1] = per[x][2 * j + 1];
        }
    return out;
}

// A device allocation [lo, hi) that GEMM operands must stay inside.
struct Extent {
    uintptr_t lo = 0, hi = 0;
};

// Result of checking a problem list against the allocations its launches use.
struct ListCheck {
    int64_t checked = 0;      // addresses and offsets checked
    int64_t violations = 0;   // of which out of their allocation or descriptor
    int64_t padding = 0;      // in-range A reads of the zero row padding (vector loads past M)
    std::string first;        // the first violation, described
    void bad(const std::string& what) {
        if (violations++ == 0) first = what;
    }
};

// Validation, longest-first order and tile ranges of a problem list (the
// order the launches and the schedule maps use).
template <class T>
int prepare_list(std::vector<GemmProblem<T>>& v) {
    // the GEMM kernel reads B as aligned (re, im) pairs
    for (const auto& P : v)
        if ((P.boff | P.ldb | P.bps | P.N) & 1) throw std::runtime_error("GEMM problem with unpaired B columns");
    // its buffer loads address one 16-row k step with 32-bit byte offsets
    // (elements of up to 8 bytes)
    for (const auto& P : v)
        if (P.lda >= (int64_t(1) << 24) || P.ldb >= (int64_t(1) << 24))
            throw std::runtime_error("GEMM row stride too large for the 32-bit offsets of the staging loads");
    std::stable_sort(v.begin(), v.end(), [](const GemmProblem<T>& x, const GemmProblem<T>& y) {
        return int64_t(x.M) * x.K > int64_t(y.M) * y.K;
    });
    return finalize_gemm_problems<T>(v.data(), int(v.size()));
}

// Extents of every problem of a finalized list against its allocations:
// A (absolute, a set-up table) must lie in one of `tables`; B and C are
// offsets from the launch's base pointers into workspace regions of
// b_bytes / c_bytes.  Cheap (per problem), run on every list a plan builds.
template <class T, class TB>
void check_extents(const std::vector<GemmProblem<T>>& v, const std::vector<Extent>& tables, size_t b_bytes,
                   size_t c_bytes, ListCheck& out) {
    for (size_t i = 0; i < v.size(); ++i) {
        const GemmProblem<T>& P = v[i];
        const std::string id = "problem " + std::to_string(i) + " (M " + std::to_string(P.M) + ", N " +
                               std::to_string(P.N) + ", K " + std::to_string(P.K) + ")";
        // A: rows 0 .. K-1 of lda elements, the last one read up to lda (vector
        // loads) or M; every k step's descriptor ends at A + (k0 + rows) lda
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(P.A);
        const uintptr_t a1 = a0 + uintptr_t(P.K) * uintptr_t(P.lda) * sizeof(T);
        bool inside = false;
        for (const Extent& e : tables) inside = inside || (a0 >= e.lo && a1 <= e.hi);
        out.checked += 1;
        if (!inside) out.bad(id + ": A rows outside every table allocation");
        // B: element (k, n) at boff + k ldb + (n >> 1) bps + (n & 1) (none when K = 0)
        const int64_t bmax = P.boff + int64_t(P.K - 1) * P.ldb + int64_t((P.N - 1) >> 1) * P.bps + 1;
        out.checked += 1;
        if (P.K > 0 && (P.boff < 0 || uint64_t(bmax + 1) * sizeof(TB) > b_bytes))
            out.bad(id + ": B outside its workspace region");
        // C: element (m, n) at coff + m ldc + (n >> 1) cps + (n & 1)
        const int64_t cmax = P.coff + int64_t(P.M - 1) * P.ldc + int64_t((P.N - 1) >> 1) * P.cps + 1;
        out.checked += 1;
        if (P.coff < 0 || uint64_t(cmax + 1) * sizeof(T) > c_bytes) out.bad(id + ": C outside its workspace region");
        // descriptor sizes stay below 2^31 (the out-of-range offset is 2^31)
        out.checked += 1;
        if (int64_t(kGemmBK) * P.lda * int64_t(sizeof(T)) >= (int64_t(1) << 31) ||
            int64_t(kGemmBK) * P.ldb * int64_t(sizeof(TB)) >= (int64_t(1) << 31))
            out.bad(id + ": descriptor records reach 2^31");
    }
}

// Replay of the GEMM kernel's staging addresses (gemm_a_offset /
// gemm_b_offset, the functions the kernel calls) for every tile of every
// problem: each element inside the problem must get an offset below its k
// step's descriptor records whose address lies in the operand's allocation,
// and each element outside (columns past M or N, rows past K) an offset at or
// past the records, so that the hardware returns zero without reading memory.
// Offsets do not depend on the k step except through its row count, so each
// tile is replayed for a full step (16 rows) and for the last step; every
// step's descriptor range is checked against the allocation.
template <class T, class TB>
void replay_list(const std::vector<GemmProblem<T>>& v, const std::vector<Extent>& tables, size_t b_bytes,
                 ListCheck& out) {
    constexpr int VE = GemmStage<T>::VE;
    for (size_t i = 0; i < v.size(); ++i) {
        const GemmProblem<T>& P = v[i];
        const std::string id = "problem " + std::to_string(i);
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(P.A);
        Extent ta{};
        for (const Extent& e : tables)
            if (a0 >= e.lo && a0 < e.hi) ta = e;
        const bool avec = gemm_a_vector(P);
        const int nk = (P.K + kGemmBK - 1) / kGemmBK;
        // every k step's descriptors inside the allocations
        for (int s = 0; s < nk; ++s) {
            const int k0 = s * kGemmBK;
            const uintptr_t abase = a0 + uintptr_t(k0) * uintptr_t(P.lda) * sizeof(T);
            const uint64_t bbase = (uint64_t(P.boff) + uint64_t(k0) * uint64_t(P.ldb)) * sizeof(TB);
            out.checked += 2;
            if (abase < ta.lo || abase + gemm_a_records(P, k0) > ta.hi)
                out.bad(id + " (M " + std::to_string(P.M) + ", K " + std::to_string(P.K) + ", lda " +
                        std::to_string(P.lda) + ", k0 " + std::to_string(k0) + "): A descriptor [" +
                        std::to_string(abase - ta.lo) + ", +" + std::to_string(gemm_a_records(P, k0)) +
                        ") outside the table of " + std::to_string(ta.hi - ta.lo) + " bytes");
            if (bbase + gemm_b_records<T, TB>(P, k0) > b_bytes)
                out.bad(id + ": B descriptor outside the workspace region");
        }
        const int tiles_m = (P.M + kGemmBM - 1) / kGemmBM;
        // a full step (if any) and the last; the kernel stages step 0 even
        // when K = 0 (no rows: every element must fall outside)
        int steps[2] = {0, nk > 0 ? (nk - 1) * kGemmBK : 0};
        const int nsteps = nk > 1 ? 2 : 1;
        for (int tm = 0; tm < tiles_m; ++tm)
            for (int tn = 0; tn < P.tiles_n; ++tn)
                for (int si = 0; si < nsteps; ++si) {
                    const int k0 = nsteps == 2 ? steps[si] : 0;
                    const int rows = gemm_step_rows(P, k0);
                    const uint32_t ra = gemm_a_records(P, k0), rb = gemm_b_records<T, TB>(P, k0);
                    const uintptr_t abase = a0 + uintptr_t(k0) * uintptr_t(P.lda) * sizeof(T);
                    const uint64_t bbase = (uint64_t(P.boff) + uint64_t(k0) * uint64_t(P.ldb)) * sizeof(TB);
                    const int m0 = tm * kGemmBM, n0 = tn * kGemmBN;
                    for (int tid = 0; tid < kGemmThreads; ++tid) {
                        const int lr = GemmStage<T>::row(tid);
                        for (int e = 0; e < 8; e += (avec ? VE : 1)) {
                            const int mm = m0 + GemmStage<T>::col(tid, e);
                            const int width = avec ? VE : 1;
                            const bool live = lr < rows && mm < P.M;   // some element of the load is in the problem
                            const uint32_t off = gemm_a_offset(P, avec, m0, tid, e);
                            out.checked += 1;
                            if (live) {
                                if (off == kGemmOOB || uint64_t(off) + width * sizeof(T) > ra ||
                                    abase + off + width * sizeof(T) > ta.hi)
                                    out.bad(id + ": A element inside the problem not read");
                                else if (mm + width > P.M)
                                    out.padding += 1;
                            } else if (off < ra && lr >= rows) {
                                out.bad(id + ": A row past K inside the descriptor");
                            } else if (off < ra) {
                                // columns past M inside the descriptor: only the
                                // zero padding of a vector-read row (mm < lda)
                                if (!(avec && mm < P.lda)) out.bad(id + ": A column past M read from memory");
                                else out.padding += 1;
                            }
                        }
                        for (int e = 0; e < 8; e += 2) {
                            const int nn = n0 + GemmStage<T>::col(tid, e);
                            const bool live = lr < rows && nn < P.N;
                            const uint32_t off = gemm_b_offset<T, TB>(P, n0, tid, e);
                            out.checked += 1;
                            if (live) {
                                if (off == kGemmOOB || uint64_t(off) + 2 * sizeof(TB) > rb ||
                                    bbase + off + 2 * sizeof(TB) > b_bytes)
                                    out.bad(id + ": B pair inside the problem not read");
                            } else if (off < rb) {
                                out.bad(id + " (N " + std::to_string(P.N) + ", K " + std::to_string(P.K) + ", ldb " +
                                        std::to_string(P.ldb) + ", bps " + std::to_string(P.bps) + ", tile n0 " +
                                        std::to_string(n0) + ", k0 " + std::to_string(k0) + ", tid " +
                                        std::to_string(tid) + ", e " + std::to_string(e) +
                                        "): B element outside the problem inside the descriptor");
                            }
                        }
                    }
                }
    }
}

template <class T>
void upload_list(std::vector<std::unique_ptr<DevBuf>>& owned, std::vector<GemmProblem<T>>& v, GemmList<T>& out) {
    out.tiles = prepare_list(v);
    out.n = int(v.size());
    out.dev = upload_int(owned, v);
    out.host = v;
    for (int c = 0; c < HP2SPH_NSCHED; ++c) {
        std::vector<int32_t> tm = c == HP2SPH_SCHED_XCD_ROUND_ROBIN ? xcd_tile_map<T>(v.data(), int(v.size()))
                                                                   : schedule_map(v, out.tiles, c);
        out.nslots[c] = int(tm.size() / 2);
        out.maps[c] = upload_int(owned, tm);
    }
    // XCD placement keeps each problem on one XCD, which leaves XCDs idle
    // when a list has fewer problems than two per XCD (the four parity-block
    // problems of the staged strategy): those start in list order, row tiles
    // of a column panel together
    out.use(v.size() < 2 * 8 ? HP2SPH_SCHED_LINEAR_ROWS : HP2SPH_SCHED_XCD_ROUND_ROBIN);
}

// Extents of a list that is about to be uploaded (throws on a violation).
template <class T, class TB = T>
void require_extents(const std::vector<GemmProblem<T>>& v, const std::vector<Extent>& tables, size_t b_bytes,
                     size_t c_bytes) {
    ListCheck c;
    check_extents<T, TB>(v, tables, b_bytes, c_bytes, c);
    if (c.violations) throw std::runtime_error("GEMM problem list out of bounds: " + c.first);
}

// Extent of a device buffer
Extent extent_of(const void* p, size_t bytes) {
    Extent e;
    e.lo = reinterpret_cast<uintptr_t>(p);
    e.hi = e.lo + bytes;
    return e;
}

// The set-up tables a staged group's GEMMs read, per block.
struct StagedBases {
    const void* ana[4] = {};        // analysis matrices [h][l'] (T)
    const double* syn[4] = {};      // synthesis matrices [l'][h]
    const double* synT[4] = {};     // their transposes [h][l'] (equal weight)
};

// TB: storage type of the Dsym rows the GEMM reads (B offsets in TB elements)
template <class T, class TB = T>
std::vector<GemmProblem<T>> staged_analysis_problems(const Group& G, const StagedBases& t) {
    const GroupDims& d = G.dims;
    std::vector<GemmProblem<T>> v;
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        GemmProblem<T> P{};
        P.A = static_cast<const T*>(t.ana[b]);
        P.M = d.nl[b];
        P.N = int(d.N[kpar]);
        P.K = 2 * G.nside + 1;
        P.lda = d.nl[b];
        P.boff = int64_t(G.blk_off_D[b] / sizeof(TB));
        P.ldb = d.N[kpar];
        P.bps = 2;
        P.coff = int64_t(G.blk_off_U[b] / sizeof(T));
        P.ldc = d.N[kpar];
        P.cps = 2;
        v.push_back(P);
    }
    return v;
}

std::vector<GemmProblem<double>> staged_synthesis_problems(const Group& G, const StagedBases& t) {
    const GroupDims& d = G.dims;
    std::vector<GemmProblem<double>> v;
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        GemmProblem<double> P{};
        P.A = t.syn[b];
        P.M = 2 * G.nside + 1;
        P.N = int(d.N[kpar]);
        P.K = d.nl[b];
        P.lda = 2 * G.nside + 1;
        P.boff = int64_t(G.blk_off_U[b] / sizeof(double));
        P.ldb = d.N[kpar];
        P.bps = 2;
        P.coff = int64_t(G.blk_off_D[b] / sizeof(double));
        P.ldc = d.N[kpar];
        P.cps = 2;
        v.push_back(P);
    }
    return v;
}

// Equal-weight analysis, staged: per block, the transposed evaluation matrix
// (rows h = 1 .. 2 nside, the rings; the pole row carries no pixel) applied to
// the weighted longitude sums, then the analysis sweeps (the transpose of the
// synthesis sweeps: the rotations are orthogonal).
std::vector<GemmProblem<double>> staged_adjoint_problems(const Group& G, const StagedBases& t) {
    const GroupDims& d = G.dims;
    std::vector<GemmProblem<double>> v;
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        GemmProblem<double> P{};
        P.A = t.synT[b] + d.nl[b];   // row h = 1
        P.M = d.nl[b];
        P.N = int(d.N[kpar]);
        P.K = 2 * G.nside;
        P.lda = d.nl[b];
        P.boff = int64_t(G.blk_off_D[b] / sizeof(double)) + d.N[kpar];
        P.ldb = d.N[kpar];
        P.bps = 2;
        P.coff = int64_t(G.blk_off_U[b] / sizeof(double));
        P.ldc = d.N[kpar];
        P.cps = 2;
        v.push_back(P);
    }
    return v;
}

// Element offsets and sizes of the per-order tables of one block.
struct OrderLayout {
    std::vector<int64_t> ana_off, syn_off, adj_off;
    std::vector<int32_t> h0;
    int64_t ana_size = 0, syn_size = 0, adj_size = 0;
};

OrderLayout order_layout(const Group& G, int b) {
    const GroupDims& d = G.dims;
    const int kpar = b >> 1, K = 2 * G.nside + 1;
    OrderLayout L;
    for (int kk = 0; kk < d.nk[b]; ++kk) {
        const int h0 = first_row(2 * kk + kpar);
        L.h0.push_back(h0);
        L.ana_off.push_back(L.ana_size);
        L.ana_size += int64_t(K - h0) * order_table_lda(d.nl[b] - kk);
        L.syn_off.push_back(L.syn_size);
        L.syn_size += int64_t(d.nl[b] - kk) * (2 * G.nside);
        L.adj_off.push_back(L.adj_size);
        L.adj_size += int64_t(2 * G.nside) * order_table_lda(d.nl[b] - kk);
    }
    return L;
}

size_t order_table_bytes(const Group& G, int mode) {
    size_t ana = 0, syn = 0, adj = 0;
    for (int b = 0; b < 4; ++b) {
        OrderLayout L = order_layout(G, b);
        ana += size_t(L.ana_size);
        syn += size_t(L.syn_size);
        adj += size_t(L.adj_size);
    }
    if (mode == HP2SPH_EQUAL_WEIGHT) return (syn + adj) * 8;
    if (mode == HP2SPH_F64) return ana * 8;
    if (mode == HP2SPH_F32) return ana * 4;
    return ana * 4 + syn * 8;
}

// Per-order tables of one group, per block (null where the mode has none).
struct OrderBases {
    const double* ana64[4] = {};
    const float* ana32[4] = {};
    const double* syn64[4] = {};
    const double* adj64[4] = {};
};

// The grouped GEMM problems of the per-order tables: one per (block, order).
struct OrderLists {
    std::vector<GemmProblem<double>> ana64, syn64, adj64;
    std::vector<GemmProblem<float>> ana32, ana32_b64;   // FP32 analysis of FP32 / FP64 ring coefficients
};

OrderLists order_problems(const Group& G, int mode, const OrderBases& t) {
    const GroupDims& d = G.dims;
    const int K = 2 * G.nside + 1;
    OrderLists out;
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        OrderLayout L = order_layout(G, b);
        for (int kk = 0; kk < d.nk[b]; ++kk) {
            // order m = p in the block whose degrees have the other parity has
            // no l: no analysis or adjoint output (no problem), while its
            // synthesis problem (K = 0) writes the zeros the ring rows need
            const bool live = d.nl[b] - kk > 0;
            const int h0 = L.h0[kk];
            // mode-major layout: mode k' of every map is one contiguous run of 2 nmaps
            const int64_t kcol = int64_t(kk) * 2 * d.nmaps;
            if (live && (t.ana64[b] || t.ana32[b])) {
                GemmProblem<double> P{};
                P.M = d.nl[b] - kk;
                P.K = K - h0;
                P.N = 2 * d.nmaps;
                P.lda = order_table_lda(P.M);
                P.ldb = d.N[kpar];
                P.bps = 2;
                P.ldc = d.N[kpar];
                P.cps = 2;
                if (mode == HP2SPH_F64) {
                    P.A = t.ana64[b] + L.ana_off[kk];
                    P.boff = int64_t(G.blk_off_D[b] / 8) + int64_t(h0) * d.N[kpar] + kcol;
                    P.coff = int64_t(G.blk_off_U[b] / 8) + int64_t(kk) * d.N[kpar] + kcol;
                    out.ana64.push_back(P);
                } else {
                    GemmProblem<float> Q{};
                    Q.A = t.ana32[b] + L.ana_off[kk];
                    Q.M = P.M;
                    Q.K = P.K;
                    Q.N = P.N;
                    Q.lda = P.lda;
                    Q.ldb = P.ldb;
                    Q.bps = P.bps;
                    Q.ldc = P.ldc;
                    Q.cps = P.cps;
                    Q.coff = int64_t(G.blk_off_U[b] / 4) + int64_t(kk) * d.N[kpar] + kcol;
                    if (mode == HP2SPH_F32_REFINE) {
                        Q.boff = int64_t(G.blk_off_D[b] / 4) + int64_t(h0) * d.N[kpar] + kcol;
                        out.ana32.push_back(Q);
                    }
                    Q.boff = int64_t(G.blk_off_D[b] / 8) + int64_t(h0) * d.N[kpar] + kcol;
                    out.ana32_b64.push_back(Q);
                }
            }
            if (t.syn64[b]) {
                GemmProblem<double> S{};
                S.A = t.syn64[b] + L.syn_off[kk];
                S.M = 2 * G.nside;
                S.K = d.nl[b] - kk;
                S.N = 2 * d.nmaps;
                S.lda = 2 * G.nside;
                S.boff = int64_t(G.blk_off_U[b] / 8) + int64_t(kk) * d.N[kpar] + kcol;
                S.ldb = d.N[kpar];
                S.bps = 2;
                S.coff = int64_t(G.blk_off_D[b] / 8) + int64_t(1) * d.N[kpar] + kcol;
                S.ldc = d.N[kpar];
                S.cps = 2;
                out.syn64.push_back(S);
            }
            if (live && t.adj64[b]) {
                // a_l^m = sum_h Tsyn[l][h] W[h]: the transposed synthesis table
                // over the ring rows h = 1 .. 2 nside
                GemmProblem<double> Q{};
                Q.A = t.adj64[b] + L.adj_off[kk];
                Q.M = d.nl[b] - kk;
                Q.K = 2 * G.nside;
                Q.N = 2 * d.nmaps;
                Q.lda = order_table_lda(Q.M);
                Q.boff = int64_t(G.blk_off_D[b] / 8) + int64_t(1) * d.N[kpar] + kcol;
                Q.ldb = d.N[kpar];
                Q.bps = 2;
                Q.coff = int64_t(G.blk_off_U[b] / 8) + int64_t(kk) * d.N[kpar] + kcol;
                Q.ldc = d.N[kpar];
                Q.cps = 2;
                out.adj64.push_back(Q);
            }
        }
    }
    return out;
}

#define HIPTHROW(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) throw std::runtime_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Build the per-order tables on the GPU: for every block and mode k', the
// analysis matrix is the analysis sweeps of column k' applied to every
// half-ring column of the fused colatitude-fit matrix; the synthesis matrix
// is the same sweeps applied to every ring row of the evaluation matrix
// (the transpose of the synthesis sweeps); the adjoint matrix of the
// equal-weight analysis is the synthesis matrix transposed.  Runs once per
// plan.
void build_order_tables(hp2sph_plan_t plan, Group& G) {
    const GroupDims& d = G.dims;
    const int K = 2 * G.nside + 1;
    const bool want_ana = (plan->mode != HP2SPH_EQUAL_WEIGHT);
    const bool want_syn = (plan->mode == HP2SPH_F32_REFINE || plan->mode == HP2SPH_EQUAL_WEIGHT);
    const bool want_adj = (plan->mode == HP2SPH_EQUAL_WEIGHT);
    OrderBases bases;
    std::vector<Extent> extents;
    // temporary buffer for the virtual batch (chains replicated over k')
    size_t per_v = 0;
    for (int b = 0; b < 4; ++b) per_v = std::max(per_v, size_t(d.nl[b]) * 2 * d.nk[b] * sizeof(double));
    const int nv_max = int(std::max<size_t>(1, std::min<size_t>((K + 1) / 2, (size_t(1) << 31) / per_v)));
    DevBuf tmp;
    tmp.bytes = per_v * nv_max;
    HIPTHROW(hipMalloc(&tmp.p, tmp.bytes));
    double* Uv = static_cast<double*>(tmp.p);
    for (int b = 0; b < 4; ++b) {
        const int kpar = b >> 1;
        OrderLayout L = order_layout(G, b);
        std::unique_ptr<DevBuf> ana64;
        if (want_ana) {
            ana64 = std::make_unique<DevBuf>();
            ana64->bytes = size_t(L.ana_size) * 8;
            HIPTHROW(hipMalloc(&ana64->p, ana64->bytes));
            HIPTHROW(hipMemset(ana64->p, 0, ana64->bytes));   // row padding reads as zero
        }
        std::unique_ptr<DevBuf> syn64;
        if (want_syn) {
            syn64 = std::make_unique<DevBuf>();
            syn64->bytes = size_t(L.syn_size) * 8;
            HIPTHROW(hipMalloc(&syn64->p, syn64->bytes));
        }
        std::vector<std::unique_ptr<DevBuf>> scratch;
        const int64_t* d_ana_off = upload_int(scratch, L.ana_off);
        const int64_t* d_syn_off = upload_int(scratch, L.syn_off);
        const int32_t* d_h0 = upload_int(scratch, L.h0);
        // dims of the virtual batch: only block b is swept
        GroupDims gv = d;
        for (int o = 0; o < 4; ++o)
            if (o != b) gv.nk[o] = 0;
        gv.nmaps = nv_max;
        gv.Npm[kpar] = 2 * d.nk[b];
        gv.N[kpar] = int64_t(nv_max) * gv.Npm[kpar];
        set_layout(gv, false);
        Blocks4<double> Ub{};
        Ub.p[b] = Uv;
        Blocks4<const double> Gv{};
        Gv.p[b] = G.t64.givens[b];
        for (int pass = 0; pass < 2; ++pass) {
            const bool syn = (pass == 1);
            if (syn ? !want_syn : !want_ana) continue;
            const int h_lo = syn ? 1 : 0, h_hi = K - 1;
            for (int hf = h_lo; hf <= h_hi; hf += 2 * nv_max) {
                if (syn) {
                    HIPTHROW(launch_replicate<double>(G.syn[b], 1, K, d.nl[b], hf, h_hi, Uv, d.nk[b], nv_max, nullptr));
                } else {
                    HIPTHROW(launch_replicate<double>(G.t64.ana[b], d.nl[b], 1, d.nl[b], hf, h_hi, Uv, d.nk[b],
                                                      nv_max, nullptr));
                }
                HIPTHROW(launch_sweep_fwd<double>(Ub, Gv, gv, nullptr));
                HIPTHROW(launch_scatter_tables<double>(Uv, d.nl[b], d.nk[b], nv_max, hf, h_hi, syn ? d_syn_off : d_ana_off,
                                                       d_h0, 2 * G.nside, syn,
                                                       static_cast<double*>(syn ? syn64->p : ana64->p), nullptr));
            }
        }
        HIPTHROW(hipDeviceSynchronize());
        std::unique_ptr<DevBuf> adj64;
        if (want_adj) {
            adj64 = std::make_unique<DevBuf>();
            adj64->bytes = size_t(L.adj_size) * 8;
            HIPTHROW(hipMalloc(&adj64->p, adj64->bytes));
            HIPTHROW(hipMemset(adj64->p, 0, adj64->bytes));   // row padding reads as zero
            const int64_t* d_adj_off = upload_int(scratch, L.adj_off);
            HIPTHROW(launch_transpose_orders(static_cast<const double*>(syn64->p), d_syn_off,
                                             static_cast<double*>(adj64->p), d_adj_off, d.nl[b], d.nk[b],
                                             2 * G.nside, nullptr));
            HIPTHROW(hipDeviceSynchronize());
        }
        if (want_ana && plan->mode != HP2SPH_F64) {
            // FP32 copy of the analysis tables (zero padding included)
            auto a32 = std::make_unique<DevBuf>();
            a32->bytes = size_t(L.ana_size) * 4;
            HIPTHROW(hipMalloc(&a32->p, a32->bytes));
            HIPTHROW(launch_convert(static_cast<const double*>(ana64->p), static_cast<float*>(a32->p), L.ana_size,
                                    nullptr));
            HIPTHROW(hipDeviceSynchronize());
            bases.ana32[b] = static_cast<const float*>(a32->p);
            extents.push_back(extent_of(a32->p, a32->bytes));
            G.owned.push_back(std::move(a32));
        } else if (want_ana) {
            bases.ana64[b] = static_cast<const double*>(ana64->p);
            extents.push_back(extent_of(ana64->p, ana64->bytes));
            G.owned.push_back(std::move(ana64));
        }
        if (want_syn) {
            bases.syn64[b] = static_cast<const double*>(syn64->p);
            extents.push_back(extent_of(syn64->p, syn64->bytes));
            G.owned.push_back(std::move(syn64));
        }
        if (want_adj) {
            bases.adj64[b] = static_cast<const double*>(adj64->p);
            extents.push_back(extent_of(adj64->p, adj64->bytes));
            G.owned.push_back(std::move(adj64));
        }
    }
    OrderLists ol = order_problems(G, plan->mode, bases);
    // every problem inside its table and its workspace regions (see the
    // launches: analysis D -> U, synthesis U -> D, adjoint D -> U)
    require_extents<double>(ol.ana64, extents, G.bytes_D, G.bytes_U);
    require_extents<float>(ol.ana32, extents, G.bytes_D, G.bytes_U);
    require_extents<float, double>(ol.ana32_b64, extents, G.bytes_D, G.bytes_U);
    require_extents<double>(ol.syn64, extents, G.bytes_U, G.bytes_D);
    require_extents<double>(ol.adj64, extents, G.bytes_D, G.bytes_U);
    if (!ol.ana64.empty()) upload_list(G.owned, ol.ana64, G.ana64);
    if (!ol.ana32.empty()) upload_list(G.owned, ol.ana32, G.ana32);
    if (!ol.ana32_b64.empty()) upload_list(G.owned, ol.ana32_b64, G.ana32_b64);
    if (!ol.syn64.empty()) upload_list(G.owned, ol.syn64, G.syn64);
    if (!ol.adj64.empty()) upload_list(G.owned, ol.adj64, G.adj64);
}

// Staged lists of one group from its device tables (extents checked, then
// uploaded).
void build_staged_lists(hp2sph_plan_t plan, Group& G) {
    const GroupDims& d = G.dims;
    const int K = 2 * G.nside + 1;
    StagedBases t64, t32;
    std::vector<Extent> ext;
    for (int b = 0; b < 4; ++b) {
        t64.ana[b] = G.t64.ana[b];
        t32.ana[b] = G.t32.ana[b];
        t64.syn[b] = G.syn[b];
        t64.synT[b] = G.synT[b];
        const size_t n = size_t(K) * d.nl[b];
        if (G.t64.ana[b]) ext.push_back(extent_of(G.t64.ana[b], n * 8));
        if (G.t32.ana[b]) ext.push_back(extent_of(G.t32.ana[b], n * 4));
        if (G.syn[b]) ext.push_back(extent_of(G.syn[b], n * 8));
        if (G.synT[b]) ext.push_back(extent_of(G.synT[b], n * 8));
    }
    auto syn = staged_synthesis_problems(G, t64);
    require_extents<double>(syn, ext, G.bytes_U, G.bytes_D);
    upload_list(G.owned, syn, G.syn64_staged);
    if (G.tables) return;
    if (plan->mode == HP2SPH_EQUAL_WEIGHT) {
        auto v = staged_adjoint_problems(G, t64);
        require_extents<double>(v, ext, G.bytes_D, G.bytes_U);
        upload_list(G.owned, v, G.adj64);
    } else if (plan->mode == HP2SPH_F64) {
        auto v = staged_analysis_problems<double>(G, t64);
        require_extents<double>(v, ext, G.bytes_D, G.bytes_U);
        upload_list(G.owned, v, G.ana64);
    } else {
        if (plan->mode == HP2SPH_F32_REFINE) {
            auto v = staged_analysis_problems<float>(G, t32);
            require_extents<float>(v, ext, G.bytes_D, G.bytes_U);
            upload_list(G.owned, v, G.ana32);
        }
        auto w = staged_analysis_problems<float, double>(G, t32);
        require_extents<float, double>(w, ext, G.bytes_D, G.bytes_U);
        upload_list(G.owned, w, G.ana32_b64);
    }
}

// Launch `expr` as stage `st`, bracketed by events when profiling is on.
#define STAGE(st, expr)                                                                        \
    do {                                                                                       \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;                                               \
        if (g_prof && g_prof->on) {                                                            \
            ea_ = g_prof->get();                                                               \
            eb_ = g_prof->get();                                                               \
            if (ea_) (void)hipEventRecord(ea_, s);                                             \
        }                                                                                      \
        HIPCHK(expr);                                                                          \
        if (ea_ && eb_) {                                                                      \
            (void)hipEventRecord(eb_, s);                                                      \
            g_prof->pending.push_back({st, ea_, eb_});                                         \
        }                                                                                      \
    } while (0)

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(HP2SPH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

template <class T>
DevTables<T>& tabs(Group& G);
template <>
DevTables<double>& tabs<double>(Group& G) { return G.t64; }
template <>
DevTables<float>& tabs<float>(Group& G) { return G.t32; }

// Work-list launch over groups [first, first + n) of the plan.
GroupLaunch span_launch(hp2sph_plan_t plan, int first, int n, void* ws, int grid_cap = 0) {
    return GroupLaunch{plan->d_gdesc, plan->gdesc.data(), first, n, static_cast<char*>(ws), grid_cap, 0};
}
GroupLaunch all_groups(hp2sph_plan_t plan, void* ws, int grid_cap = 0) {
    return span_launch(plan, 0, int(plan->groups.size()), ws, grid_cap);
}
// The ring-transform launch over groups [first, first + n), with the plan's
// item order.
GroupLaunch ring_launch(hp2sph_plan_t plan, int first, int n, void* ws) {
    GroupLaunch gl = span_launch(plan, first, n, ws);
    gl.variant = plan->ring_order;
    gl.threads = plan->ring_threads;
    return gl;
}
// The pack launch over groups [first, first + n), with the plan's tile shape.
GroupLaunch pack_launch(hp2sph_plan_t plan, int first, int n, void* ws) {
    GroupLaunch gl = span_launch(plan, first, n, ws);
    gl.variant = plan->pack_maps;
    return gl;
}

// S1 of every group into region `reg`: one launch per span of groups that
// share the ring kernels' thread count.
int ring_forward_all(hp2sph_plan_t plan, const double* maps, int reg, void* ws, hipStream_t s) {
    for (const auto& sp : plan->ring_spans)
        STAGE(0, launch_ring_forward(maps, ring_launch(plan, sp.first, sp.second, ws), reg, s));
    return HP2SPH_OK;
}

template <class T>
const GemmList<T>& merged_analysis(const hp2sph_plan_s* plan);
template <>
const GemmList<double>& merged_analysis<double>(const hp2sph_plan_s* plan) { return plan->m_ana64; }
template <>
const GemmList<float>& merged_analysis<float>(const hp2sph_plan_s* plan) { return plan->m_ana32_b64; }

// One analysis of every group, colatitude fit and conversion in precision T:
// maps -> alm.  Each stage is one work-list launch over all groups (the
// GEMM one launch over the merged problem list); the Givens sweeps of groups
// on the staged strategy run per group.  The ring transform and pole values
// are FP64 in both precisions (for T = float this is the first pass of the
// refinement: the GEMM rounds the FP64 ring coefficients to FP32 as it
// stages them).
template <class T>
int analysis_all(hp2sph_plan_t plan, const double* maps, double* alm, void* ws, hipStream_t s) {
    if (int e = ring_forward_all(plan, maps, kRegD, ws, s)) return e;
    STAGE(1, launch_pole<double>(all_groups(plan, ws), kRegD, s));
    const GemmList<T>& gl = merged_analysis<T>(plan);
    STAGE(2, (launch_gemm<T, double>(gl.dev, gl.tmap, gl.slots, static_cast<const double*>(ws), static_cast<T*>(ws),
                                     s)));
    for (auto& gp : plan->groups) {
        Group& G = *gp;
        if (G.tables) continue;
        Blocks4<const T> Gv;
        for (int b = 0; b < 4; ++b) Gv.p[b] = tabs<T>(G).givens[b];
        STAGE(3, launch_sweep_fwd<T>(blocks_at<T>(ws, G.off_U, G, G.rows_U), Gv, G.dims, s));
    }
    STAGE(4, launch_pack<T>(pack_launch(plan, 0, int(plan->groups.size()), ws), kRegU, -1, alm, s));
    return HP2SPH_OK;
}

// FP64 synthesis of one group up to the ring coefficients: alm -> Dsym rows
// 1 .. 2 nside of the D region (D+- of every mode k = 0..p per ring pair).
int synthesis_coefficients(Group& G, const double* alm, void* ws, hipStream_t s) {
    Blocks4<double> D = blocks_at<double>(ws, G.off_D, G, G.rows_D);
    Blocks4<double> U = blocks_at<double>(ws, G.off_U, G, G.rows_U);
    const bool tab = G.syn64.n > 0 && G.tables;
    // the staged synthesis sweeps need the map-major column order, whatever
    // the group uses for its analysis
    GroupDims dd = G.dims;
    if (!tab) set_layout(dd, false);
    STAGE(5, launch_unpack(alm, G.d_alm_off, G.d_lmax, U, dd, s));
    if (!tab) {
        Blocks4<const double> Gv;
        for (int b = 0; b < 4; ++b) Gv.p[b] = G.t64.givens[b];
        STAGE(6, launch_sweep_bwd<double>(U, Gv, dd, s));
    }
    const GemmList<double>& gl = tab ? G.syn64 : G.syn64_staged;
    STAGE(7, launch_gemm<double>(gl.dev, gl.tmap, gl.slots, U.p[0], D.p[0], s));
    return HP2SPH_OK;
}

// FP64 synthesis of one group: alm -> out (or minus_from - synthesis).
int synthesis_pass(Group& G, const double* alm, double* out, const double* minus_from, void* ws, hipStream_t s) {
    if (int e = synthesis_coefficients(G, alm, ws, s)) return e;
    Blocks4<double> D = blocks_at<double>(ws, G.off_D, G, G.rows_D);
    GroupDims dd = G.dims;
    if (!(G.syn64.n > 0 && G.tables)) set_layout(dd, false);
    STAGE(8, launch_ring_inverse(cblocks(D), G.rings, G.t64.fft, out, minus_from, G.d_map_off, dd, s));
    return HP2SPH_OK;
}

// FP32 analysis with one FP64 refinement (Sec. 2.2, eq. uzawa, with A the
// FP32 analysis and S the FP64 synthesis), every group at once:
//   a0 = A32 f,  a1 = a0 + A32 (f - S a0).
// The residual is formed after the ring transform, which is linear:
// Ring(f - S a0) = Ring(f) - Ring(S a0).  Ring(f) is computed once in FP64;
// Ring(S a0) is the synthesis GEMM output folded onto each ring's modes
// (k_residual_fold), exactly what an inverse and a forward ring FFT would
// give, without the two transforms.  The residual enters the FP32 stages
// rounded to FP32 (FP32 colatitude fit and Legendre conversion).
int refine_all(hp2sph_plan_t plan, const double* maps, double* alm, void* ws, hipStream_t s) {
    auto staged_sweeps = [&](int region, bool fwd) -> int {
        for (auto& gp : plan->groups) {
            Group& G = *gp;
            if (G.tables) continue;
            if (fwd) {
                Blocks4<const float> Gv32;
                for (int b = 0; b < 4; ++b) Gv32.p[b] = G.t32.givens[b];
                const size_t off = region == kRegUa ? G.off_Ua : G.off_U;
                STAGE(3, launch_sweep_fwd<float>(blocks_at<float>(ws, off, G, G.rows_U), Gv32, G.dims, s));
            } else {
                Blocks4<const double> Gv;
                for (int b = 0; b < 4; ++b) Gv.p[b] = G.t64.givens[b];
                STAGE(6, launch_sweep_bwd<double>(blocks_at<double>(ws, G.off_U, G, G.rows_U), Gv, G.dims, s));
            }
        }
        return HP2SPH_OK;
    };
    const double* wsd = static_cast<const double*>(ws);
    // a0 = A32 f: FP64 ring coefficients (region Df), rounded to FP32 as the
    // GEMM stages them; a0 in region Ua
    if (int e = ring_forward_all(plan, maps, kRegDf, ws, s)) return e;
    STAGE(1, launch_pole<double>(all_groups(plan, ws), kRegDf, s));
    const GemmList<float>& gb = plan->m_ana32_b64;
    STAGE(2, (launch_gemm<float, double>(gb.dev, gb.tmap, gb.slots, wsd, static_cast<float*>(ws), s)));
    if (int e = staged_sweeps(kRegUa, true)) return e;
    // S a0 up to the inverse ring transform (FP64): a0 widened to FP64 (and
    // truncated at each map's lmax) into region U, then the synthesis GEMM
    // into region D
    STAGE(5, launch_widen(all_groups(plan, ws), s));
    if (int e = staged_sweeps(kRegU, false)) return e;
    const GemmList<double>& gs = plan->m_syn64;
    STAGE(7, launch_gemm<double>(gs.dev, gs.tmap, gs.slots, wsd, static_cast<double*>(ws), s));
    // residual ring coefficients (region Dr), the correction A32 r (region
    // U), and a1 = a0 + A32 r
    STAGE(10, launch_residual_fold(all_groups(plan, ws, plan->fold_grid), s));
    STAGE(1, launch_pole<float>(all_groups(plan, ws), kRegDr, s));
    const GemmList<float>& ga = plan->m_ana32;
    STAGE(2, launch_gemm<float>(ga.dev, ga.tmap, ga.slots, static_cast<const float*>(ws), static_cast<float*>(ws), s));
    if (int e = staged_sweeps(kRegU, true)) return e;
    STAGE(4, launch_pack<float>(pack_launch(plan, 0, int(plan->groups.size()), ws), kRegUa, kRegU, alm, s));
    return HP2SPH_OK;
}

// Equal-weight analysis of one group, eq. (healsph) (Sec. 2.2), from weighted
// longitude sums W (Dsym rows 1 .. 2 nside, see launch_ring_adjoint):
// a = sum_h Tsyn[l][h] W[h], the synthesis transposed -- the transposed
// evaluation tables and (staged) the analysis sweeps.  Written to alm, or
// added to it (the update of the Jacobi iteration).
int equal_weight_apply(hp2sph_plan_t plan, Group& G, Blocks4<double> W, double* alm, bool add, void* ws,
                       hipStream_t s) {
    Blocks4<double> U = blocks_at<double>(ws, G.off_U, G, G.rows_U);
    STAGE(12, launch_gemm<double>(G.adj64.dev, G.adj64.tmap, G.adj64.slots, W.p[0], U.p[0], s));
    if (!G.tables) {
        Blocks4<const double> Gv;
        for (int b = 0; b < 4; ++b) Gv.p[b] = G.t64.givens[b];
        STAGE(3, launch_sweep_fwd<double>(U, Gv, G.dims, s));
    }
    if (add) {
        Blocks4<double> Ua = blocks_at<double>(ws, G.off_Ua, G, G.rows_U);
        STAGE(5, launch_unpack(alm, G.d_alm_off, G.d_lmax, Ua, G.dims, s));
        STAGE(4, launch_pack<double>(pack_launch(plan, G.index, 1, ws), kRegUa, kRegU, alm, s));
    } else {
        STAGE(4, launch_pack<double>(pack_launch(plan, G.index, 1, ws), kRegU, -1, alm, s));
    }
    return HP2SPH_OK;
}

// The Jacobi iteration of eq. (uzawa) with A = (4 pi / N) S^* (Sec. 2.2):
// a0 = A f, then niter times r = f - S a, a = a + A r (all FP64).  A is
// linear and starts with the longitude sums, so A r = A' (Wf - W(S a)) with
// Wf = W(f) computed once and W(S a) formed from the synthesis coefficients
// (k_adjoint_residual): the residual map is never materialised.
int jacobi_pass(hp2sph_plan_t plan, Group& G, const double* maps, double* alm, int niter, void* ws, hipStream_t s) {
    Blocks4<double> Wf = blocks_at<double>(ws, G.off_Wf, G, G.rows_D);
    Blocks4<double> Wr = blocks_at<double>(ws, G.off_Wr, G, G.rows_D);
    Blocks4<double> Gs = blocks_at<double>(ws, G.off_D, G, G.rows_D);
    const double scale = 4.0 * 3.14159265358979323846 / (12.0 * double(G.nside) * double(G.nside));
    STAGE(11, launch_ring_adjoint(maps, G.d_map_off, G.rings, G.t64.fft, Wf, G.dims, scale, s));
    if (G.tables) {
        // per-order tables: a stays in the U layout both GEMMs use (truncated
        // at each map's lmax) and is packed once at the end
        Blocks4<double> U = blocks_at<double>(ws, G.off_U, G, G.rows_U);
        Blocks4<double> Ua = blocks_at<double>(ws, G.off_Ua, G, G.rows_U);
        STAGE(12, launch_gemm<double>(G.adj64.dev, G.adj64.tmap, G.adj64.slots, Wf.p[0], U.p[0], s));
        STAGE(5, launch_accumulate(cblocks(U), Ua, G.d_lmax, G.dims, true, s));
        for (int it = 0; it < niter; ++it) {
            STAGE(7, launch_gemm<double>(G.syn64.dev, G.syn64.tmap, G.syn64.slots, Ua.p[0], Gs.p[0], s));
            STAGE(10, launch_adjoint_residual(cblocks(Wf), cblocks(Gs), Wr, G.rings, G.dims, scale, s));
            STAGE(12, launch_gemm<double>(G.adj64.dev, G.adj64.tmap, G.adj64.slots, Wr.p[0], U.p[0], s));
            STAGE(5, launch_accumulate(cblocks(U), Ua, G.d_lmax, G.dims, false, s));
        }
        STAGE(4, launch_pack<double>(pack_launch(plan, G.index, 1, ws), kRegUa, -1, alm, s));
        return HP2SPH_OK;
    }
    if (int e = equal_weight_apply(plan, G, Wf, alm, false, ws, s)) return e;
    for (int it = 0; it < niter; ++it) {
        if (int e = synthesis_coefficients(G, alm, ws, s)) return e;
        STAGE(10, launch_adjoint_residual(cblocks(Wf), cblocks(Gs), Wr, G.rings, G.dims, scale, s));
        if (int e = equal_weight_apply(plan, G, Wr, alm, true, ws, s)) return e;
    }
    return HP2SPH_OK;
}

// Byte offset and size of region r of a group.
std::pair<size_t, size_t> region_span(const Group& G, int r) {
    switch (r) {
        case kRegD: return {G.off_D, G.bytes_D};
        case kRegU: return {G.off_U, G.bytes_U};
        case kRegDf: return {G.off_Df, G.bytes_D};
        case kRegDr: return {G.off_Dr, G.bytes_D};
        default: return {G.off_Ua, G.bytes_U};
    }
}

// The problems one role's GEMM runs for every group, moved from their
// group's region bases (B in region breg, C in region creg) to the workspace
// base, into one list: one launch then serves all groups, its problems
// sorted longest first across groups.  Every rebased problem is checked to
// stay inside its group's regions (the per-group lists were checked against
// the region sizes when they were built).
template <class T, class TB, class Pick>
void merge_role(hp2sph_plan_t plan, Pick pick, int breg, int creg, GemmList<T>& out) {
    std::vector<GemmProblem<T>> v;
    for (auto& gp : plan->groups) {
        Group& G = *gp;
        const GemmList<T>* L = pick(G);
        if (!L || L->host.empty()) continue;
        const auto bsp = region_span(G, breg);
        const auto csp = region_span(G, creg);
        for (GemmProblem<T> P : L->host) {
            P.boff += int64_t(bsp.first / sizeof(TB));
            P.coff += int64_t(csp.first / sizeof(T));
            const int64_t bmax = P.boff + int64_t(P.K - 1) * P.ldb + int64_t((P.N - 1) >> 1) * P.bps + 1;
            const int64_t cmax = P.coff + int64_t(P.M - 1) * P.ldc + int64_t((P.N - 1) >> 1) * P.cps + 1;
            const bool b_in = P.K == 0 || (uint64_t(P.boff) * sizeof(TB) >= bsp.first &&
                                           uint64_t(bmax + 1) * sizeof(TB) <= bsp.first + bsp.second);
            const bool c_in = uint64_t(P.coff) * sizeof(T) >= csp.first &&
                              uint64_t(cmax + 1) * sizeof(T) <= csp.first + csp.second;
            if (!b_in || !c_in) throw std::runtime_error("merged GEMM problem outside its group's workspace regions");
            v.push_back(P);
        }
    }
    if (!v.empty()) upload_list(plan->owned, v, out);
}

// Device descriptors of the groups (regions at their final offsets), the
// ring kernels' spans, the merged GEMM lists of the analysis and the
// batch-wide per-map arrays.  Run once the workspace layout is fixed.
void build_work_lists(hp2sph_plan_t plan) {
    const int mode = plan->mode;
    plan->gdesc.clear();
    for (auto& gp : plan->groups) {
        const Group& G = *gp;
        GroupDesc d{};
        d.g = G.dims;
        d.rt = G.rings;
        d.ft = G.t64.fft;
        d.map_off = G.d_map_off;
        d.alm_off = G.d_alm_off;
        d.lmax = G.d_lmax;
        if (G.dims.modemajor) {
            d.pack_tiles = G.d_pack_tiles;
            d.n_pack_tiles = G.n_pack_tiles;
        } else {
            std::vector<int32_t> pt = pack_tiles_mapmajor(G.dims.p);
            d.n_pack_tiles = int(pt.size() / 2);
            d.pack_tiles = upload_int(plan->owned, pt);
        }
        d.tables = G.tables ? 1 : 0;
        for (int i = 0; i < 3; ++i) d.pole_w[i] = G.pole_w[i];
        for (int r = 0; r < kRegions; ++r)
            for (int b = 0; b < 4; ++b) d.reg[r][b] = -1;
        const bool has_df = mode == HP2SPH_F32_REFINE, has_ua = has_df || mode == HP2SPH_EQUAL_WEIGHT;
        for (int b = 0; b < 4; ++b) {
            d.reg[kRegD][b] = int64_t(G.off_D + G.blk_off_D[b]);
            d.reg[kRegU][b] = int64_t(G.off_U + G.blk_off_U[b]);
            if (has_df) {
                d.reg[kRegDf][b] = int64_t(G.off_Df + G.blk_off_D[b]);
                d.reg[kRegDr][b] = int64_t(G.off_Dr + G.blk_off_D[b]);
            }
            if (has_ua) d.reg[kRegUa][b] = int64_t(G.off_Ua + G.blk_off_U[b]);
        }
        plan->gdesc.push_back(d);
    }
    plan->d_gdesc = upload_int(plan->owned, plan->gdesc);
    // spans of consecutive groups (descending nside) whose ring kernels run
    // the same thread count
    plan->ring_spans.clear();
    for (int i = 0; i < int(plan->groups.size()); ++i) {
        const int nt = ring_threads(plan->gdesc[i].ft.fft_max);
        if (!plan->ring_spans.empty()) {
            auto& last = plan->ring_spans.back();
            if (ring_threads(plan->gdesc[last.first].ft.fft_max) == nt && last.second < kMaxGroups) {
                ++last.second;
                continue;
            }
        }
        plan->ring_spans.push_back({i, 1});
    }
    switch (mode) {
        case HP2SPH_F64:
            merge_role<double, double>(plan, [](Group& G) { return &G.ana64; }, kRegD, kRegU, plan->m_ana64);
            break;
        case HP2SPH_F32:
            merge_role<float, double>(plan, [](Group& G) { return &G.ana32_b64; }, kRegD, kRegU, plan->m_ana32_b64);
            break;
        case HP2SPH_F32_REFINE:
            merge_role<float, double>(plan, [](Group& G) { return &G.ana32_b64; }, kRegDf, kRegUa,
                                      plan->m_ana32_b64);
            merge_role<double, double>(plan, [](Group& G) { return G.tables ? &G.syn64 : &G.syn64_staged; }, kRegU,
                                       kRegD, plan->m_syn64);
            merge_role<float, float>(plan, [](Group& G) { return &G.ana32; }, kRegDr, kRegU, plan->m_ana32);
            break;
        default:
            break;   // the equal-weight analysis runs per group
    }
    std::vector<int64_t> ao(plan->alm_off.begin(), plan->alm_off.end()), co(plan->cl_off.begin(), plan->cl_off.end());
    plan->d_alm_off = upload_int(plan->owned, ao);
    plan->d_cl_off = upload_int(plan->owned, co);
    plan->d_lmax = upload_int(plan->owned, plan->lmax);
    plan->lmax_max = 0;
    for (int32_t l : plan->lmax) plan->lmax_max = std::max(plan->lmax_max, int(l));
}

// ---------------------------------------------------------------------------
// Tuning cache: the autotuner's choices keyed by plan shape
// ---------------------------------------------------------------------------
//
// Key: the device's architecture and compute-unit count, the mode and, per
// group, nside, number of maps and strategy.  Value: the schedule of every
// tuned GEMM (in the order hp2sph_schedules reports them), the fold's work
// grid, the pack's tile shape and the ring transform's item order.  Kept per process; HP2SPH_TUNE_CACHE names a text file that is read
// once and appended to (one "key = values" line per entry, the last line of
// a key wins), so tuned shapes start tuned in later processes too.

struct TuneChoice {
    std::vector<int> sched;
    int fold_grid = 0;
    int pack_maps = 32;
    int ring_order = 0;
    int ring_threads = 256;
};

std::mutex g_tune_mu;
std::map<std::string, TuneChoice>& tune_cache() {
    static std::map<std::string, TuneChoice> m;
    return m;
}
bool g_tune_file_read = false;

int device_cus(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

std::string tune_key(const hp2sph_plan_s* plan) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, plan->device) == hipSuccess) arch = prop.gcnArchName;
    // "v2": entries hold the fold grid, pack tile, ring order, ring threads,
    // then the GEMM schedules
    std::string k = "v2/" + arch + "/" + std::to_string(device_cus(plan->device)) + "/mode" +
                    std::to_string(plan->mode);
    for (const auto& g : plan->groups)
        k += "/" + std::to_string(g->nside) + "x" + std::to_string(g->dims.nmaps) + (g->tables ? "t" : "s");
    return k;
}

void read_tune_file_locked() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = std::getenv("HP2SPH_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        const size_t eq = l.find(" = ");
        if (eq == std::string::npos) continue;
        TuneChoice c;
        std::vector<long> v;
        const char* q = l.c_str() + eq + 3;
        char* end = nullptr;
        for (long x = std::strtol(q, &end, 10); end != q; x = std::strtol(q, &end, 10)) {
            v.push_back(x);
            q = end;
        }
        if (v.size() < 4) continue;
        c.fold_grid = int(v[0]);
        c.pack_maps = int(v[1]);
        c.ring_order = int(v[2]);
        c.ring_threads = int(v[3]);
        for (size_t i = 4; i < v.size(); ++i) c.sched.push_back(int(v[i]));
        tune_cache()[l.substr(0, eq)] = c;
    }
    std::fclose(f);
}

void store_tune(const hp2sph_plan_s* plan, const TuneChoice& c) {
    const std::string key = tune_key(plan);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file_locked();
    tune_cache()[key] = c;
    const char* path = std::getenv("HP2SPH_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE* f = std::fopen(path, "a")) {
        std::string line = key + " = " + std::to_string(c.fold_grid) + " " + std::to_string(c.pack_maps) + " " +
                           std::to_string(c.ring_order) + " " + std::to_string(c.ring_threads);
        for (int x : c.sched) line += " " + std::to_string(x);
        line += "\n";
        std::fputs(line.c_str(), f);
        std::fclose(f);
    }
}

bool lookup_tune(const hp2sph_plan_s* plan, TuneChoice& c) {
    const std::string key = tune_key(plan);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file_locked();
    auto it = tune_cache().find(key);
    if (it == tune_cache().end()) return false;
    c = it->second;
    return true;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Handles of the plans that are alive (created and not yet destroyed).  A
// handle is checked against this set before anything reads through it, so a
// destroyed or never-created handle gives ESTATE without touching its memory.
std::mutex g_plans_mu;
std::unordered_set<const hp2sph_plan_s*>& live_plans() {
    static std::unordered_set<const hp2sph_plan_s*> s;
    return s;
}

int check_plan(hp2sph_plan_t plan) {
    if (!plan) return fail(HP2SPH_ESTATE, "plan handle is null");
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!live_plans().count(plan)) return fail(HP2SPH_ESTATE, "not a live plan handle (never created, or destroyed)");
    return HP2SPH_OK;
}

int check_workspace(hp2sph_plan_t plan, const void* workspace, size_t bytes) {
    if (!workspace || !aligned(workspace, kAlign)) return fail(HP2SPH_EWORKSPACE, "workspace null or not 256-byte aligned");
    if (bytes < plan->ws_bytes)
        return fail(HP2SPH_EWORKSPACE, "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                                           std::to_string(plan->ws_bytes) + " bytes the plan needs");
    return HP2SPH_OK;
}

// The grouped GEMMs hp2sph_analyze launches, in launch order: the merged
// lists of the analysis modes, or each group's lists of the equal-weight
// analysis.
void analysis_lists(hp2sph_plan_t plan, std::vector<GemmSched*>& out) {
    auto add = [&](GemmSched& L, int n) {
        if (n > 0) out.push_back(&L);
    };
    switch (plan->mode) {
        case HP2SPH_F64: add(plan->m_ana64, plan->m_ana64.n); break;
        case HP2SPH_F32: add(plan->m_ana32_b64, plan->m_ana32_b64.n); break;
        case HP2SPH_F32_REFINE:
            add(plan->m_ana32_b64, plan->m_ana32_b64.n);
            add(plan->m_syn64, plan->m_syn64.n);
            add(plan->m_ana32, plan->m_ana32.n);
            break;
        default:   // equal weight: transposed evaluation, then the synthesis of each iteration
            for (auto& g : plan->groups) {
                Group& G = *g;
                GemmList<double>& syn = G.tables ? G.syn64 : G.syn64_staged;
                add(G.adj64, G.adj64.n);
                add(syn, syn.n);
            }
            break;
    }
}

// Every GEMM list the plan built (merged and per group).
void built_lists(hp2sph_plan_t plan, std::vector<GemmSched*>& out) {
    for (GemmSched* L : {static_cast<GemmSched*>(&plan->m_ana64), static_cast<GemmSched*>(&plan->m_syn64),
                         static_cast<GemmSched*>(&plan->m_ana32_b64), static_cast<GemmSched*>(&plan->m_ana32)})
        if (L->maps[0]) out.push_back(L);
    for (auto& g : plan->groups) {
        Group& G = *g;
        for (GemmSched* L : {static_cast<GemmSched*>(&G.ana64), static_cast<GemmSched*>(&G.syn64),
                             static_cast<GemmSched*>(&G.syn64_staged), static_cast<GemmSched*>(&G.adj64),
                             static_cast<GemmSched*>(&G.ana32), static_cast<GemmSched*>(&G.ana32_b64)})
            if (L->maps[0]) out.push_back(L);
    }
}

}  // namespace

extern "C" {

const char* hp2sph_last_error(void) { return g_last_error.c_str(); }

int hp2sph_plan_create(const int32_t* nside, const int32_t* lmax, int32_t batch, int32_t mode,
                       hp2sph_plan_t* out) {
    return hp2sph_plan_create_ex(nside, lmax, batch, mode, HP2SPH_STRATEGY_AUTO, out);
}

int hp2sph_plan_create_ex(const int32_t* nside, const int32_t* lmax, int32_t batch, int32_t mode, int32_t strategy,
                          hp2sph_plan_t* out) {
    if (!out) return fail(HP2SPH_EINVAL, "out is null");
    *out = nullptr;
    if (!nside || !lmax) return fail(HP2SPH_EINVAL, "nside/lmax is null");
    if (batch <= 0) return fail(HP2SPH_EINVAL, "batch must be positive");
    if (mode != HP2SPH_F64 && mode != HP2SPH_F32_REFINE && mode != HP2SPH_F32 && mode != HP2SPH_EQUAL_WEIGHT)
        return fail(HP2SPH_EINVAL, "unknown precision mode");
    if (strategy != HP2SPH_STRATEGY_AUTO && strategy != HP2SPH_STRATEGY_STAGED && strategy != HP2SPH_STRATEGY_TABLES)
        return fail(HP2SPH_EINVAL, "unknown strategy");
    for (int b = 0; b < batch; ++b) {
        if (nside[b] < 2 || nside[b] > HP2SPH_MAX_NSIDE || !is_pow2(nside[b]))
            return fail(HP2SPH_EINVAL, "nside must be a power of two in [2, " + std::to_string(HP2SPH_MAX_NSIDE) + "]");
        if (lmax[b] < 0 || lmax[b] > 2 * nside[b]) return fail(HP2SPH_EINVAL, "need 0 <= lmax <= 2 nside");
    }
    std::unique_ptr<hp2sph_plan_s> plan;
    try {
        plan.reset(new hp2sph_plan_s());
        plan->batch = batch;
        plan->mode = mode;
        plan->strategy = strategy;
        if (hipGetDevice(&plan->device) != hipSuccess) return fail(HP2SPH_EDEVICE, "hipGetDevice failed");
        plan->nside.assign(nside, nside + batch);
        plan->lmax.assign(lmax, lmax + batch);
        int64_t mo = 0, ao = 0, co = 0;
        for (int b = 0; b < batch; ++b) {
            plan->map_off.push_back(mo);
            plan->alm_off.push_back(ao);
            plan->cl_off.push_back(co);
            mo += 12LL * nside[b] * nside[b];
            ao += int64_t(lmax[b] + 1) * (lmax[b] + 2) / 2;
            co += lmax[b] + 1;
        }
        plan->total_pix = mo;
        plan->total_alm = ao;
        plan->total_cl = co;
        std::map<int, std::vector<int>> bys;
        for (int b = 0; b < batch; ++b) bys[nside[b]].push_back(b);
        for (auto it = bys.rbegin(); it != bys.rend(); ++it) {
            auto G = std::make_unique<Group>();
            G->nside = it->first;
            G->members = it->second;
            init_dims(*G);
            // strategy: per-order tables when asked, or (auto) when the batch is
            // large enough to fill MFMA tiles and the tables take at most a
            // quarter of the device memory (and fit in what is free); staged
            // sweeps otherwise
            bool tables = (strategy == HP2SPH_STRATEGY_TABLES);
            size_t fre = 0, tot = 0;
            if (hipMemGetInfo(&fre, &tot) != hipSuccess) return fail(HP2SPH_EDEVICE, "hipMemGetInfo failed");
            if (strategy == HP2SPH_STRATEGY_AUTO) {
                const size_t need = order_table_bytes(*G, mode);
                tables = G->dims.nmaps >= 8 && need <= tot / 4 && need <= fre;
            }
            // tables that cannot fit are refused before anything is built or
            // allocated for them
            if (tables && order_table_bytes(*G, mode) > fre)
                return fail(HP2SPH_ENOMEM, "per-order tables of nside " + std::to_string(G->nside) + " need " +
                                               std::to_string(order_table_bytes(*G, mode) >> 20) + " MiB, " +
                                               std::to_string(fre >> 20) + " MiB of device memory are free");
            build_group(plan.get(), *G);
            G->tables = tables;
            set_layout(G->dims, tables);
            build_staged_lists(plan.get(), *G);
            if (tables) build_order_tables(plan.get(), *G);
            G->index = int(plan->groups.size());
            plan->groups.push_back(std::move(G));
        }
        if (int(plan->groups.size()) > kMaxGroups) return fail(HP2SPH_EINVAL, "too many distinct nside values");
        // workspace: every group its own regions, back to back
        size_t ws = 0;
        auto take = [&](size_t bytes) {
            const size_t at = ws;
            ws += align_up(bytes);
            return at;
        };
        for (auto& g : plan->groups) {
            Group& G = *g;
            G.off_D = take(G.bytes_D);
            G.off_U = take(G.bytes_U);
            if (mode == HP2SPH_F32_REFINE) {
                G.off_Df = take(G.bytes_D);
                G.off_Dr = take(G.bytes_D);
                G.off_Ua = take(G.bytes_U);
            } else if (mode == HP2SPH_EQUAL_WEIGHT) {
                G.off_Ua = take(G.bytes_U);
                G.off_Wf = take(G.bytes_D);
                G.off_Wr = take(G.bytes_D);
            }
        }
        build_work_lists(plan.get());
        plan->ws_bytes = ws;
        // a shape the autotuner has seen (in this process, or in the
        // HP2SPH_TUNE_CACHE file) starts with its choices
        {
            TuneChoice c;
            if (lookup_tune(plan.get(), c)) {
                std::vector<GemmSched*> lists;
                analysis_lists(plan.get(), lists);
                if (c.sched.size() == lists.size()) {
                    for (size_t i = 0; i < lists.size(); ++i)
                        if (c.sched[i] >= 0 && c.sched[i] < HP2SPH_NSCHED) lists[i]->use(c.sched[i]);
                    plan->fold_grid = c.fold_grid;
                    if (c.pack_maps == 16 || c.pack_maps == 32 || c.pack_maps == 64) plan->pack_maps = c.pack_maps;
                    if (c.ring_order >= 0 && c.ring_order <= 2) plan->ring_order = c.ring_order;
                    if (c.ring_threads == 256 || c.ring_threads == 512) plan->ring_threads = c.ring_threads;
                }
            }
        }
        // kernels with more than 64 KB of dynamic LDS
        if (configure_kernels() != hipSuccess) return fail(HP2SPH_EDEVICE, "hipFuncSetAttribute failed");
        // device address of this device's static workspace (for
        // hp2sph_analyze_noalloc), looked up once per device at set-up
        if (hipError_t e = scratch_init(); e != hipSuccess)
            return fail(HP2SPH_EDEVICE, std::string("hipGetSymbolAddress of the static workspace: ") +
                                            hipGetErrorString(e));
    } catch (const std::bad_alloc&) {
        return fail(HP2SPH_ENOMEM, "allocation of plan tables failed");
    } catch (const std::exception& e) {
        return fail(HP2SPH_EDEVICE, e.what());
    }
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        live_plans().insert(plan.get());
    }
    *out = plan.release();
    return HP2SPH_OK;
}

int hp2sph_plan_strategy(hp2sph_plan_t plan, int32_t* strategy) {
    if (int e = check_plan(plan)) return e;
    if (!strategy) return fail(HP2SPH_EINVAL, "strategy is null");
    int nt = 0;
    for (auto& g : plan->groups) nt += g->tables ? 1 : 0;
    *strategy = (nt == 0) ? HP2SPH_STRATEGY_STAGED
                          : (nt == int(plan->groups.size()) ? HP2SPH_STRATEGY_TABLES : HP2SPH_STRATEGY_AUTO);
    return HP2SPH_OK;
}

int hp2sph_workspace_size(hp2sph_plan_t plan, size_t* bytes) {
    if (int e = check_plan(plan)) return e;
    if (!bytes) return fail(HP2SPH_EINVAL, "bytes is null");
    *bytes = plan->ws_bytes;
    return HP2SPH_OK;
}

int hp2sph_analyze(hp2sph_plan_t plan, const double* maps, double* alm, void* workspace, size_t workspace_bytes,
                   void* stream) {
    if (int e = check_plan(plan)) return e;
    g_prof = &plan->prof;
    if (!maps || !alm) return fail(HP2SPH_EINVAL, "maps/alm is null");
    if (!aligned(maps, 16) || !aligned(alm, 16)) return fail(HP2SPH_EINVAL, "maps/alm not 16-byte aligned");
    if (int e = check_workspace(plan, workspace, workspace_bytes)) return e;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (plan->mode) {
        case HP2SPH_F64: return analysis_all<double>(plan, maps, alm, workspace, s);
        case HP2SPH_F32: return analysis_all<float>(plan, maps, alm, workspace, s);
        case HP2SPH_F32_REFINE: return refine_all(plan, maps, alm, workspace, s);
        default:
            for (auto& gp : plan->groups)
                if (int e = jacobi_pass(plan, *gp, maps, alm, kDefaultJacobi, workspace, s)) return e;
            return HP2SPH_OK;
    }
}

static_assert(kScratchBytes == HP2SPH_NOALLOC_WORKSPACE, "static workspace size of the C ABI");

int hp2sph_analyze_noalloc(hp2sph_plan_t plan, const double* maps, double* alm, void* stream) {
    if (int e = check_plan(plan)) return e;
    if (plan->ws_bytes > kScratchBytes)
        return fail(HP2SPH_EINVAL, "the plan needs " + std::to_string(plan->ws_bytes) + " bytes of workspace, more than "
                                   "the " + std::to_string(kScratchBytes) + " bytes of the static workspace");
    void* ws = scratch_ptr(plan->device);
    if (!ws) return fail(HP2SPH_ESTATE, "no static workspace on the plan's device");
    // no profiling events here: they come from a pool that may need creating
    Profiler* const saved = g_prof;
    const bool was_on = plan->prof.on;
    plan->prof.on = false;
    const int e = hp2sph_analyze(plan, maps, alm, ws, kScratchBytes, stream);
    plan->prof.on = was_on;
    g_prof = saved;
    return e;
}

int hp2sph_analyze_iterative(hp2sph_plan_t plan, const double* maps, double* alm, int32_t niter, void* workspace,
                             size_t workspace_bytes, void* stream) {
    if (int e = check_plan(plan)) return e;
    g_prof = &plan->prof;
    if (plan->mode != HP2SPH_EQUAL_WEIGHT) return fail(HP2SPH_EINVAL, "plan was not created with HP2SPH_EQUAL_WEIGHT");
    if (niter < 0 || niter > HP2SPH_MAX_JACOBI) return fail(HP2SPH_EINVAL, "niter out of range");
    if (!maps || !alm) return fail(HP2SPH_EINVAL, "maps/alm is null");
    if (!aligned(maps, 16) || !aligned(alm, 16)) return fail(HP2SPH_EINVAL, "maps/alm not 16-byte aligned");
    if (int e = check_workspace(plan, workspace, workspace_bytes)) return e;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (auto& gp : plan->groups)
        if (int e = jacobi_pass(plan, *gp, maps, alm, niter, workspace, s)) return e;
    return HP2SPH_OK;
}

int hp2sph_synthesize(hp2sph_plan_t plan, const double* alm, double* maps, void* workspace, size_t workspace_bytes,
                      void* stream) {
    if (int e = check_plan(plan)) return e;
    g_prof = &plan->prof;
    if (!maps || !alm) return fail(HP2SPH_EINVAL, "maps/alm is null");
    if (!aligned(maps, 16) || !aligned(alm, 16)) return fail(HP2SPH_EINVAL, "maps/alm not 16-byte aligned");
    if (int e = check_workspace(plan, workspace, workspace_bytes)) return e;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (auto& gp : plan->groups)
        if (int e = synthesis_pass(*gp, alm, maps, nullptr, workspace, s)) return e;
    return HP2SPH_OK;
}

int hp2sph_power_spectrum(hp2sph_plan_t plan, const double* alm, double* cl, void* stream) {
    if (int e = check_plan(plan)) return e;
    g_prof = &plan->prof;
    if (!alm || !cl) return fail(HP2SPH_EINVAL, "alm/cl is null");
    if (!aligned(alm, 16) || !aligned(cl, 8)) return fail(HP2SPH_EINVAL, "alm/cl misaligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    STAGE(9, launch_cl(alm, plan->d_alm_off, plan->d_lmax, cl, plan->d_cl_off, plan->batch, plan->lmax_max, s));
    return HP2SPH_OK;
}

int hp2sph_profile(hp2sph_plan_t plan, int32_t enable) {
    if (int e = check_plan(plan)) return e;
    if (hipError_t e = plan->prof.drain(); e != hipSuccess) return fail(HP2SPH_EDEVICE, hipGetErrorString(e));
    if (enable) {
        for (int i = 0; i < HP2SPH_NSTAGES; ++i) {
            plan->prof.ms[i] = 0.0;
            plan->prof.launches[i] = 0;
        }
    }
    plan->prof.on = enable != 0;
    return HP2SPH_OK;
}

int hp2sph_profile_read(hp2sph_plan_t plan, double* ms, int32_t* launches, int32_t nstages) {
    if (int e = check_plan(plan)) return e;
    if (!ms || !launches || nstages < 0 || nstages > HP2SPH_NSTAGES) return fail(HP2SPH_EINVAL, "bad arguments");
    if (hipError_t e = plan->prof.drain(); e != hipSuccess) return fail(HP2SPH_EDEVICE, hipGetErrorString(e));
    for (int i = 0; i < nstages; ++i) {
        ms[i] = plan->prof.ms[i];
        launches[i] = plan->prof.launches[i];
    }
    return HP2SPH_OK;
}

int hp2sph_set_schedule(hp2sph_plan_t plan, int32_t sched) {
    if (int e = check_plan(plan)) return e;
    if (sched < 0 || sched >= HP2SPH_NSCHED) return fail(HP2SPH_EINVAL, "unknown schedule");
    std::vector<GemmSched*> lists;
    built_lists(plan, lists);
    for (GemmSched* L : lists) L->use(sched);
    return HP2SPH_OK;
}

int hp2sph_schedules(hp2sph_plan_t plan, int32_t* out, int32_t cap, int32_t* count) {
    if (int e = check_plan(plan)) return e;
    if (!count || cap < 0 || (cap > 0 && !out)) return fail(HP2SPH_EINVAL, "bad arguments");
    std::vector<GemmSched*> lists;
    analysis_lists(plan, lists);
    for (int i = 0; i < int(lists.size()) && i < cap; ++i) out[i] = lists[i]->sched;
    *count = int(lists.size());
    return HP2SPH_OK;
}

int hp2sph_set_option(hp2sph_plan_t plan, int32_t option, int32_t value) {
    if (int e = check_plan(plan)) return e;
    switch (option) {
        case HP2SPH_OPT_FOLD_GRID:
            if (value < 0 || (value > 0 && value < 8))
                return fail(HP2SPH_EINVAL, "the fold grid is 0 or at least 8 workgroups");
            plan->fold_grid = value / 8 * 8;
            return HP2SPH_OK;
        case HP2SPH_OPT_PACK_MAPS:
            if (value != 16 && value != 32 && value != 64) return fail(HP2SPH_EINVAL, "maps per pack tile: 16, 32 or 64");
            plan->pack_maps = value;
            return HP2SPH_OK;
        case HP2SPH_OPT_RING_ORDER:
            if (value < 0 || value > 2) return fail(HP2SPH_EINVAL, "ring item order: 0, 1 or 2");
            plan->ring_order = value;
            return HP2SPH_OK;
        case HP2SPH_OPT_RING_THREADS:
            if (value != 256 && value != 512) return fail(HP2SPH_EINVAL, "ring transform threads: 256 or 512");
            plan->ring_threads = value;
            return HP2SPH_OK;
        default: return fail(HP2SPH_EINVAL, "unknown option");
    }
}

int hp2sph_get_option(hp2sph_plan_t plan, int32_t option, int32_t* value) {
    if (int e = check_plan(plan)) return e;
    if (!value) return fail(HP2SPH_EINVAL, "null output");
    switch (option) {
        case HP2SPH_OPT_FOLD_GRID: *value = plan->fold_grid; return HP2SPH_OK;
        case HP2SPH_OPT_PACK_MAPS: *value = plan->pack_maps; return HP2SPH_OK;
        case HP2SPH_OPT_RING_ORDER: *value = plan->ring_order; return HP2SPH_OK;
        case HP2SPH_OPT_RING_THREADS: *value = plan->ring_threads; return HP2SPH_OK;
        default: return fail(HP2SPH_EINVAL, "unknown option");
    }
}

int hp2sph_autotune(hp2sph_plan_t plan, const double* maps, double* alm, void* workspace, size_t workspace_bytes,
                    void* stream, int32_t reps, double* best_ms) {
    if (int e = check_plan(plan)) return e;
    if (reps < 1 || reps > HP2SPH_MAX_TUNE_REPS) return fail(HP2SPH_EINVAL, "reps out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool prof_on = plan->prof.on;
    // restores the profiler and frees the events on every exit
    struct Cleanup {
        hp2sph_plan_t plan;
        bool prof_on;
        hipEvent_t* ev;
        ~Cleanup() {
            plan->prof.on = prof_on;
            for (int i = 0; i < 2; ++i)
                if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    } cleanup{plan, prof_on, ev};
    if (int e = hp2sph_profile(plan, 0)) return e;
    for (int i = 0; i < 2; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) return fail(HP2SPH_EDEVICE, "hipEventCreate failed");
    // fastest of reps analyses, after an untimed one
    auto timed = [&](double& ms) -> int {
        if (int e = hp2sph_analyze(plan, maps, alm, workspace, workspace_bytes, stream)) return e;
        ms = 1e300;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(ev[0], s) != hipSuccess) return fail(HP2SPH_EDEVICE, "hipEventRecord failed");
            if (int e = hp2sph_analyze(plan, maps, alm, workspace, workspace_bytes, stream)) return e;
            float f = 0.f;
            if (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                hipEventElapsedTime(&f, ev[0], ev[1]) != hipSuccess)
                return fail(HP2SPH_EDEVICE, "timing events failed");
            ms = std::min(ms, double(f));
        }
        return HP2SPH_OK;
    };
    std::vector<GemmSched*> lists;
    analysis_lists(plan, lists);
    double best = 0.0;
    if (int e = timed(best)) return e;
    for (GemmSched* L : lists) {
        int keep = L->sched;
        for (int c = 0; c < HP2SPH_NSCHED; ++c) {
            if (c == keep) continue;
            const int prev = L->sched;
            L->use(c);
            double t = 0.0;
            if (int e = timed(t)) {
                L->use(prev);
                return e;
            }
            if (t < best * (1.0 - 0.005)) {
                best = t;
                keep = c;
            }
            L->use(keep);
        }
    }
    // work grid of the refinement's fold: one workgroup per work item, or a
    // persistent grid of 2 or 4 workgroups per compute unit walking the list
    if (plan->mode == HP2SPH_F32_REFINE) {
        const int cus = device_cus(plan->device);
        const int cand[3] = {0, 2 * cus, 4 * cus};
        int keep = plan->fold_grid;
        for (int c : cand) {
            if (c == keep) continue;
            plan->fold_grid = c;
            double t = 0.0;
            if (int e = timed(t)) {
                plan->fold_grid = keep;
                return e;
            }
            if (t < best * (1.0 - 0.005)) {
                best = t;
                keep = c;
            }
            plan->fold_grid = keep;
        }
    }
    // tile shape of the pack (maps per tile), item order and thread count of
    // the ring transform (512 threads only changes groups up to nside 1024)
    bool small_rings = false;
    for (const auto& d : plan->gdesc) small_rings = small_rings || ring_threads(d.ft.fft_max) == 256;
    for (int which = 0; which < 3; ++which) {
        if (which >= 1 && plan->mode == HP2SPH_EQUAL_WEIGHT) break;   // no forward ring transform there
        if (which == 2 && !small_rings) break;
        int& opt = which == 0 ? plan->pack_maps : which == 1 ? plan->ring_order : plan->ring_threads;
        const std::vector<int> cand = which == 0   ? std::vector<int>{32, 16, 64}
                                      : which == 1 ? std::vector<int>{0, 1, 2}
                                                   : std::vector<int>{256, 512};
        int keep = opt;
        for (int c : cand) {
            if (c == keep) continue;
            opt = c;
            double t = 0.0;
            if (int e = timed(t)) {
                opt = keep;
                return e;
            }
            if (t < best * (1.0 - 0.005)) {
                best = t;
                keep = c;
            }
            opt = keep;
        }
    }
    {
        TuneChoice c;
        for (GemmSched* L : lists) c.sched.push_back(L->sched);
        c.fold_grid = plan->fold_grid;
        c.pack_maps = plan->pack_maps;
        c.ring_order = plan->ring_order;
        c.ring_threads = plan->ring_threads;
        store_tune(plan, c);
    }
    // leave alm holding the analysis under the chosen schedules
    if (int e = hp2sph_analyze(plan, maps, alm, workspace, workspace_bytes, stream)) return e;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(HP2SPH_EDEVICE, "hipStreamSynchronize failed");
    if (best_ms) *best_ms = best;
    return HP2SPH_OK;
}

int hp2sph_plan_destroy(hp2sph_plan_t plan) {
    if (!plan) return fail(HP2SPH_ESTATE, "plan handle is null");
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        if (live_plans().erase(plan) == 0)
            return fail(HP2SPH_ESTATE, "not a live plan handle (never created, or destroyed)");
    }
    delete plan;
    return HP2SPH_OK;
}

int hp2sph_schedule_map(int32_t sched, const int32_t* M, const int32_t* N, const int32_t* K, int32_t n,
                        int32_t* out, int64_t capacity, int64_t* count) {
    if (!count) return fail(HP2SPH_EINVAL, "count is null");
    if (sched < 0 || sched >= HP2SPH_NSCHED) return fail(HP2SPH_EINVAL, "unknown schedule");
    if (n < 0 || (n > 0 && (!M || !N || !K))) return fail(HP2SPH_EINVAL, "bad problem list");
    if (capacity < 0 || (capacity > 0 && !out)) return fail(HP2SPH_EINVAL, "bad output buffer");
    std::vector<int32_t> map;
    try {
        std::vector<GemmProblem<double>> v(static_cast<size_t>(n), GemmProblem<double>{});
        for (int i = 0; i < n; ++i) {
            if (M[i] <= 0 || N[i] <= 0 || K[i] <= 0) return fail(HP2SPH_EINVAL, "non-positive problem size");
            v[i].M = M[i];
            v[i].N = N[i];
            v[i].K = K[i];
        }
        const int tiles = finalize_gemm_problems<double>(v.data(), n);
        map = sched == HP2SPH_SCHED_XCD_ROUND_ROBIN ? xcd_tile_map<double>(v.data(), n) : schedule_map(v, tiles, sched);
    } catch (const std::bad_alloc&) {
        return fail(HP2SPH_ENOMEM, "host allocation failed");
    }
    *count = int64_t(map.size());
    if (capacity > 0)
        std::memcpy(out, map.data(), sizeof(int32_t) * size_t(std::min<int64_t>(capacity, int64_t(map.size()))));
    return HP2SPH_OK;
}

int hp2sph_gemm_check(int32_t nside, int32_t nmaps, int32_t mode, int32_t strategy, int64_t* checked,
                      int64_t* violations, int64_t* padding) {
    if (!checked || !violations || !padding) return fail(HP2SPH_EINVAL, "null output");
    if (nside < 2 || nside > HP2SPH_MAX_NSIDE || !is_pow2(nside)) return fail(HP2SPH_EINVAL, "bad nside");
    if (nmaps < 1) return fail(HP2SPH_EINVAL, "nmaps must be positive");
    if (mode < HP2SPH_F64 || mode > HP2SPH_EQUAL_WEIGHT) return fail(HP2SPH_EINVAL, "unknown precision mode");
    if (strategy != HP2SPH_STRATEGY_STAGED && strategy != HP2SPH_STRATEGY_TABLES)
        return fail(HP2SPH_EINVAL, "strategy must be staged or tables");
    ListCheck c;
    try {
        Group G;
        G.nside = nside;
        for (int i = 0; i < nmaps; ++i) G.members.push_back(i);
        init_dims(G);
        const bool tables = strategy == HP2SPH_STRATEGY_TABLES;
        G.tables = tables;
        set_layout(G.dims, tables);
        // stand-in addresses for the device tables: disjoint 256-byte aligned
        // ranges of the sizes the plan allocates (nothing is dereferenced)
        uintptr_t next = uintptr_t(1) << 40;
        std::vector<Extent> ext;
        auto place = [&](size_t bytes) {
            Extent e = extent_of(reinterpret_cast<const void*>(next), bytes);
            ext.push_back(e);
            next += (bytes + 4095) / 4096 * 4096 + 4096;
            return reinterpret_cast<const void*>(e.lo);
        };
        const int K = 2 * nside + 1;
        auto run = [&](auto v, auto tb_tag, size_t b_bytes, size_t c_bytes) {
            using T = std::remove_cv_t<std::remove_pointer_t<decltype(v[0].A)>>;
            using TB = decltype(tb_tag);
            prepare_list(v);
            check_extents<T, TB>(v, ext, b_bytes, c_bytes, c);
            replay_list<T, TB>(v, ext, b_bytes, c);
        };
        if (!tables) {
            StagedBases t;
            for (int b = 0; b < 4; ++b) {
                const size_t n = size_t(K) * G.dims.nl[b];
                t.ana[b] = place(n * (mode == HP2SPH_F64 ? 8 : 4));
                t.syn[b] = static_cast<const double*>(place(n * 8));
                t.synT[b] = static_cast<const double*>(place(n * 8));
            }
            run(staged_synthesis_problems(G, t), double{}, G.bytes_U, G.bytes_D);
            if (mode == HP2SPH_EQUAL_WEIGHT) run(staged_adjoint_problems(G, t), double{}, G.bytes_D, G.bytes_U);
            else if (mode == HP2SPH_F64) run(staged_analysis_problems<double>(G, t), double{}, G.bytes_D, G.bytes_U);
            else {
                if (mode == HP2SPH_F32_REFINE) run(staged_analysis_problems<float>(G, t), float{}, G.bytes_D, G.bytes_U);
                run(staged_analysis_problems<float, double>(G, t), double{}, G.bytes_D, G.bytes_U);
            }
        } else {
            OrderBases t;
            for (int b = 0; b < 4; ++b) {
                OrderLayout L = order_layout(G, b);
                if (mode == HP2SPH_F64) t.ana64[b] = static_cast<const double*>(place(size_t(L.ana_size) * 8));
                if (mode == HP2SPH_F32 || mode == HP2SPH_F32_REFINE)
                    t.ana32[b] = static_cast<const float*>(place(size_t(L.ana_size) * 4));
                if (mode == HP2SPH_F32_REFINE || mode == HP2SPH_EQUAL_WEIGHT)
                    t.syn64[b] = static_cast<const double*>(place(size_t(L.syn_size) * 8));
                if (mode == HP2SPH_EQUAL_WEIGHT) t.adj64[b] = static_cast<const double*>(place(size_t(L.adj_size) * 8));
            }
            OrderLists ol = order_problems(G, mode, t);
            if (!ol.ana64.empty()) run(ol.ana64, double{}, G.bytes_D, G.bytes_U);
            if (!ol.ana32.empty()) run(ol.ana32, float{}, G.bytes_D, G.bytes_U);
            if (!ol.ana32_b64.empty()) run(ol.ana32_b64, double{}, G.bytes_D, G.bytes_U);
            if (!ol.syn64.empty()) run(ol.syn64, double{}, G.bytes_U, G.bytes_D);
            if (!ol.adj64.empty()) run(ol.adj64, double{}, G.bytes_D, G.bytes_U);
        }
    } catch (const std::bad_alloc&) {
        return fail(HP2SPH_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(HP2SPH_EINVAL, e.what());
    }
    *checked = c.checked;
    *violations = c.violations;
    *padding = c.padding;
    g_last_error = c.violations ? c.first : std::string();
    return HP2SPH_OK;
}

int hp2sph_host_table(int32_t nside, int32_t table, int32_t block, double* out, int64_t capacity, int64_t* count) {
    if (!count) return fail(HP2SPH_EINVAL, "count is null");
    if (nside < 2 || nside > HP2SPH_MAX_NSIDE || !is_pow2(nside)) return fail(HP2SPH_EINVAL, "bad nside");
    if (table < HP2SPH_TABLE_RINGS || table > HP2SPH_TABLE_GIVENS) return fail(HP2SPH_EINVAL, "bad table");
    if ((table >= HP2SPH_TABLE_ANALYSIS) && (block < 0 || block > 3)) return fail(HP2SPH_EINVAL, "bad block");
    std::vector<double> v;
    try {
        HostTables h;
        if (table == HP2SPH_TABLE_RINGS) {
            const int nr = 4 * nside - 1;
            int64_t st = 0;
            for (int r = 1; r <= nr; ++r) {
                RingGeom g = ring_geom(nside, r);
                v.push_back(g.z);
                v.push_back(double(g.n));
                v.push_back(g.phi0);
                v.push_back(double(st));
                st += g.n;
            }
        } else {
            build_tables(nside, h, false);
            if (table == HP2SPH_TABLE_POLE) v.assign(h.pole_w, h.pole_w + 3);
            else if (table == HP2SPH_TABLE_ANALYSIS) v = h.ana[block];
            else if (table == HP2SPH_TABLE_SYNTHESIS) v = h.syn[block];
            else {
                BlockShape bs = block_shape(nside, block);
                const int T = bs.nsweep, nl = bs.nl;
                v.assign(size_t(std::max(T, 0)) * nl * 2, 0.0);
                for (int t = 0; t < T; ++t)
                    for (int lp = 0; lp < nl; ++lp) {
                        v[(size_t(t) * nl + lp) * 2] = h.givens[block][(size_t(lp) * T + t) * 2];
                        v[(size_t(t) * nl + lp) * 2 + 1] = h.givens[block][(size_t(lp) * T + t) * 2 + 1];
                    }
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(HP2SPH_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(HP2SPH_EINVAL, e.what());
    }
    *count = int64_t(v.size());
    if (out) std::memcpy(out, v.data(), sizeof(double) * size_t(std::min<int64_t>(capacity, int64_t(v.size()))));
    return HP2SPH_OK;
}

}  // extern "C"
