// Device kernels of libhp2sph (gfx950).  See kernels.h for the data layout.
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace hp2sph {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------

template <class T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

template <class T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }
template <class T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
template <class T>
__device__ __forceinline__ C2<T> ldc(const T* p, int64_t i) { return {p[2 * i], p[2 * i + 1]}; }

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

struct alignas(16) D2 {
    double x, y;
};
struct alignas(8) F2 {
    float x, y;
};

// LDS slot of FFT entry i: one pad slot every 16 entries, so that the
// strided accesses of the Stockham passes spread over the banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Multiplication by e^{-2 pi i q / 16}, q = 0..7, with the exact forms for
// q = 0, 2, 4, 6.
template <class T, int Q>
__device__ __forceinline__ C2<T> rot16(C2<T> a) {
    constexpr T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    constexpr T h = T(0.70710678118654752440);
    if constexpr (Q == 0) return a;
    else if constexpr (Q == 1) return {c1 * a.x + s1 * a.y, c1 * a.y - s1 * a.x};
    else if constexpr (Q == 2) return {h * (a.x + a.y), h * (a.y - a.x)};
    else if constexpr (Q == 3) return {s1 * a.x + c1 * a.y, s1 * a.y - c1 * a.x};
    else if constexpr (Q == 4) return {a.y, -a.x};
    else if constexpr (Q == 5) return {c1 * a.y - s1 * a.x, -s1 * a.y - c1 * a.x};
    else if constexpr (Q == 6) return {h * (a.y - a.x), -h * (a.x + a.y)};
    else return {s1 * a.y - c1 * a.x, -c1 * a.y - s1 * a.x};
}

template <int R>
constexpr int rev_bits(int v) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (v & 1);
        v >>= 1;
    }
    return r;
}

// One butterfly stage (half-length H) of an in-register radix-2 DIT FFT of
// size R over bit-reversed input; recursion over the positions keeps every
// twiddle a compile-time constant.
template <class T, int R, int H, int POS>
__device__ __forceinline__ void dit_stage_pos(C2<T>* v) {
    if constexpr (POS < H) {
#pragma unroll
        for (int g = 0; g < R; g += 2 * H) {
            const C2<T> u = v[g + POS];
            const C2<T> t = rot16<T, POS * (8 / H)>(v[g + POS + H]);
            v[g + POS] = cadd(u, t);
            v[g + POS + H] = csub(u, t);
        }
        dit_stage_pos<T, R, H, POS + 1>(v);
    }
}

template <class T, int R, int H>
__device__ __forceinline__ void dit_stages(C2<T>* v) {
    if constexpr (H < R) {
        dit_stage_pos<T, R, H, 0>(v);
        dit_stages<T, R, 2 * H>(v);
    }
}

// In-register DFT of size R (2, 4, 8 or 16), e^{-2 pi i r s / R}, natural
// order in and out.
template <class T, int R>
__device__ __forceinline__ void dft_regs(C2<T>* v) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = rev_bits<R>(i);
        if (r > i) {
            const C2<T> t = v[i];
            v[i] = v[r];
            v[r] = t;
        }
    }
    dit_stages<T, R, 1>(v);
}

// The LDS buffer as the input of a pass (entry i at slot lpad(i)).
template <class T>
struct LdsLoad {
    const C2<T>* buf;
    __device__ __forceinline__ C2<T> operator()(int i) const { return buf[lpad(i)]; }
};

// One Stockham pass of radix R over M points with NT threads: group j reads
// entries j + r M/R (from `load`), multiplies entry r by w^r with
// w = e^{-2 pi i (j mod Ns) / (Ns R)}, transforms, and stores output r at
// (j / Ns) Ns R + (j mod Ns) + r Ns of the LDS buffer.  After the last pass
// the buffer holds the DFT in natural order.  Reads complete (barrier) before
// any thread writes, so the pass may read the buffer it writes.  The NT
// threads are threadIdx.x mod NT: a workgroup of 2 NT threads can run two
// transforms of the same length side by side (every thread meets every
// barrier).
//
// LDS addressing: when Ns is 1 or a multiple of 16 (radix-16 passes, and
// every radix-8 pass but the second), an output run base + r Ns sits at
// lpad(base) + r s with s = 1 (Ns = 1: base is a multiple of R, which
// divides 16, so base + r never crosses a pad) or s = 17 Ns / 16 (after a
// first radix-8 pass, Ns = 8, each output takes its own slot); likewise the inputs j + r G of an LDS pass sit at
// lpad(j) + r 17 G / 16 when G = M / R is a multiple of 16 (M >= 256).  The
// slot of entry r is then one base address plus a stride, and with the
// transform length a template argument (MS > 0; 0: known at run time) the
// strides are immediate offsets of the LDS instructions.
// Twiddles w, w^2, w^4, w^8 of each of a thread's groups in one pass,
// loaded ahead of the pass (a pass of a transform whose length is a
// template argument gets them from the pass before it, so the table loads
// are in flight across that pass instead of stalling this one).
template <class T, int R, int MAXV>
struct PassTw {
    C2<T> w[MAXV / R][4];
};

template <class T, int R, int NT, int MAXV>
__device__ __forceinline__ void load_pass_tw(PassTw<T, R, MAXV>& t, const T* tw, int fft_max, int lgNs, int G) {
    const int Ns = 1 << lgNs;
#pragma unroll
    for (int i = 0; i < MAXV / R; ++i) {
        const int j = (threadIdx.x & (NT - 1)) + NT * i;
        if (j < G) {
            const int st = (fft_max >> lgNs) / R * (j & (Ns - 1));
            t.w[i][0] = ldc(tw, st);
            if constexpr (R > 2) t.w[i][1] = ldc(tw, 2 * st);
            if constexpr (R > 4) t.w[i][2] = ldc(tw, 4 * st);
            if constexpr (R > 8) t.w[i][3] = ldc(tw, 8 * st);
        }
    }
}

template <class T, int R, int NT, int MAXV, int MS, bool PRE = false, class Load>
__device__ __forceinline__ void stockham_pass(C2<T>* buf, int M_rt, int lgNs, const T* tw, int fft_max, Load load,
                                              const PassTw<T, R, MAXV>& pre = PassTw<T, R, MAXV>{}) {
    constexpr int NG = MAXV / R;
    const int M = MS > 0 ? MS : M_rt;
    const int G = M / R, Ns = 1 << lgNs;
    constexpr bool lds_in = std::is_same<Load, LdsLoad<T>>::value;
    const bool linear_in = lds_in && (MS > 0 ? (MS / R) % 16 == 0 : M >= 256);
    const int sin_ = G + (G >> 4);                     // input stride (slots) when linear
    const int sout = Ns == 1 ? 1 : Ns + (Ns >> 4);      // output stride (slots)
    C2<T> v[MAXV];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int j = (threadIdx.x & (NT - 1)) + NT * i;
        if (j < G) {
            if (linear_in) {
                const C2<T>* src = buf + lpad(j);
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = src[r * sin_];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = load(j + r * G);
            }
            if (lgNs > 0) {
                // w^r, r = 1..R-1, w = e^{-2 pi i (j mod Ns) / (Ns R)}: the
                // powers 1, 2, 4, 8 from the table, the others as products of
                // two or three of them (a few ulp)
                C2<T> w[R];
                if constexpr (PRE) {
                    w[1] = pre.w[i][0];
                    if constexpr (R > 2) w[2] = pre.w[i][1];
                    if constexpr (R > 4) w[4] = pre.w[i][2];
                    if constexpr (R > 8) w[8] = pre.w[i][3];
                } else {
                    const int st = (fft_max >> lgNs) / R * (j & (Ns - 1));
                    w[1] = ldc(tw, st);
                    if constexpr (R > 2) w[2] = ldc(tw, 2 * st);
                    if constexpr (R > 4) w[4] = ldc(tw, 4 * st);
                    if constexpr (R > 8) w[8] = ldc(tw, 8 * st);
                }
                if constexpr (R > 3) w[3] = cmul(w[2], w[1]);
                if constexpr (R > 4) {
                    w[5] = cmul(w[4], w[1]);
                    w[6] = cmul(w[4], w[2]);
                    w[7] = cmul(w[4], w[3]);
                }
                if constexpr (R > 8) {
#pragma unroll
                    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], w[r]);
            }
            dft_regs<T, R>(v + i * R);
        }
    }
    __syncthreads();
    const bool linear_out = Ns == 1 || (Ns & 15) == 0;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int j = (threadIdx.x & (NT - 1)) + NT * i;
        if (j < G) {
            const int base = ((j >> lgNs) << lgNs) * R + (j & (Ns - 1));
            if (linear_out) {
                C2<T>* dst = buf + lpad(base);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * sout] = v[i * R + r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) buf[lpad(base + r * Ns)] = v[i * R + r];
            }
        }
    }
    __syncthreads();
}

template <class T, int NT, int MAXV, int MS, class Load>
__device__ __forceinline__ void stockham_dispatch(int bits, C2<T>* buf, int M, int lgNs, const T* tw, int fft_max,
                                                  Load load) {
    switch (bits) {
        case 4:
            if constexpr (MAXV >= 16) stockham_pass<T, 16, NT, MAXV, MS>(buf, M, lgNs, tw, fft_max, load);
            break;
        case 3: stockham_pass<T, 8, NT, MAXV, MS>(buf, M, lgNs, tw, fft_max, load); break;
        case 2: stockham_pass<T, 4, NT, MAXV, MS>(buf, M, lgNs, tw, fft_max, load); break;
        default: stockham_pass<T, 2, NT, MAXV, MS>(buf, M, lgNs, tw, fft_max, load); break;
    }
}

// Forward DFT of M = 2^e points (2 <= M <= NT * MAXV) in LDS, with M a
// template argument (MS > 0) or known at run time (MS = 0):
// X_s = sum_q x_q e^{-2 pi i q s / M}.  The first pass takes its input from
// `load0(q)` (which may read the buffer); on return the buffer holds X in
// natural order at slots lpad(s).  Passes of radix 16 (8 when a thread holds
// MAXV = 8 values), the remainder last.
// Table tw: e^{-2 pi i t / fft_max}, t < fft_max, M divides fft_max.
constexpr int static_log2(int v) { return v <= 1 ? 0 : 1 + static_log2(v >> 1); }
// log2 of the radix of the full passes with MAXV values per thread.
constexpr int radix_bits(int maxv) { return maxv >= 16 ? 4 : 3; }
// Radix of pass p of a transform of 2^E points: 2^RB, the remainder last.
constexpr int pass_radix(int E, int p, int RB) {
    return p < (E + RB - 1) / RB - 1 ? (1 << RB) : (1 << (E - RB * ((E + RB - 1) / RB - 1)));
}

template <class T, int NT, int MAXV, int MS, class Load0>
__device__ __forceinline__ void fft_lds_n(C2<T>* buf, int M_rt, const T* tw, int fft_max, Load0 load0) {
    const LdsLoad<T> lds_load{buf};
    constexpr int RB = radix_bits(MAXV);
    if constexpr (MS > 0) {
        // compile-time pass sequence; each pass prefetches the twiddles of
        // the next one (full passes, and a last pass of radix 8 or less)
        constexpr int E = static_log2(MS), P = (E + RB - 1) / RB;
        static_assert(P <= 4, "at most four passes");
        constexpr int R0 = pass_radix(E, 0, RB), R1 = pass_radix(E, 1, RB), R2 = pass_radix(E, 2, RB),
                      R3 = pass_radix(E, 3, RB);
        constexpr bool pre1 = P > 1 && R1 >= 8, pre2 = P > 2 && R2 >= 8, pre3 = P > 3 && R3 >= 8;
        PassTw<T, R1, MAXV> t1;
        if constexpr (pre1) load_pass_tw<T, R1, NT, MAXV>(t1, tw, fft_max, RB, MS / R1);
        stockham_pass<T, R0, NT, MAXV, MS>(buf, MS, 0, tw, fft_max, load0);
        if constexpr (P > 1) {
            PassTw<T, R2, MAXV> t2;
            if constexpr (pre2) load_pass_tw<T, R2, NT, MAXV>(t2, tw, fft_max, 2 * RB, MS / R2);
            stockham_pass<T, R1, NT, MAXV, MS, pre1>(buf, MS, RB, tw, fft_max, lds_load, t1);
            if constexpr (P > 2) {
                PassTw<T, R3, MAXV> t3;
                if constexpr (pre3) load_pass_tw<T, R3, NT, MAXV>(t3, tw, fft_max, 3 * RB, MS / R3);
                stockham_pass<T, R2, NT, MAXV, MS, pre2>(buf, MS, 2 * RB, tw, fft_max, lds_load, t2);
                if constexpr (P > 3)
                    stockham_pass<T, R3, NT, MAXV, MS, pre3>(buf, MS, 3 * RB, tw, fft_max, lds_load, t3);
            }
        }
    } else {
        const int M = M_rt;
        const int e = ilog2(M);
        const int P = (e + RB - 1) / RB;
        const int last = e - RB * (P - 1);
        // straight-line pass sequence (at most 4 passes: M <= 2^16, or 2^12
        // with radix-8 passes)
        stockham_dispatch<T, NT, MAXV, MS>(P == 1 ? last : RB, buf, M, 0, tw, fft_max, load0);
        if (P > 1) stockham_dispatch<T, NT, MAXV, MS>(P == 2 ? last : RB, buf, M, RB, tw, fft_max, lds_load);
        if (P > 2) stockham_dispatch<T, NT, MAXV, MS>(P == 3 ? last : RB, buf, M, 2 * RB, tw, fft_max, lds_load);
        if (P > 3) stockham_dispatch<T, NT, MAXV, MS>(last, buf, M, 3 * RB, tw, fft_max, lds_load);
    }
}

// fft_lds_n with the length NT * MAXV / 2 (the transforms of the equatorial
// rings and the half-buffer transforms) and NT * MAXV (the largest Bluestein
// transforms) compiled for their length.
template <class T, int NT, int MAXV, class Load0>
__device__ __forceinline__ void fft_lds(C2<T>* buf, int M, const T* tw, int fft_max, Load0 load0) {
    constexpr int kFull = NT * MAXV;
    if (M == kFull) fft_lds_n<T, NT, MAXV, kFull>(buf, M, tw, fft_max, load0);
    else if (M == kFull / 2) fft_lds_n<T, NT, MAXV, kFull / 2>(buf, M, tw, fft_max, load0);
    else fft_lds_n<T, NT, MAXV, 0>(buf, M, tw, fft_max, load0);
}

// Forward DFT of length L (a power of two, or any L through Bluestein's
// chirp-z with M = M_blue points) of the sequence src(q), q < L.  On return
// Z(k), k < L, gives output k (valid until the buffer is rewritten).
template <class T>
struct DftOut {
    const C2<T>* buf;
    const T* chirp;   // null for a direct transform
    T invM;
    __device__ C2<T> Z(int k) const {
        const C2<T> b = buf[lpad(k)];
        if (!chirp) return b;
        return cmul(ldc(chirp, k), cscale(cconj(b), invM));
    }
};

template <class T, int NT, int MAXV, class Src>
__device__ __forceinline__ DftOut<T> ring_dft(C2<T>* buf, int L, int M_blue, const T* chirp, const T* chirpfft, const T* tw,
                              int fft_max, Src src) {
    if (M_blue == 0) {
        fft_lds<T, NT, MAXV>(buf, L, tw, fft_max, src);
        return {buf, nullptr, T(1)};
    }
    // y_q = src(q) w_q (zero padded to M), Y = FFT(y), then the inverse FFT of
    // Y . FFT(conj w) through conj(FFT(conj(.))).
    fft_lds<T, NT, MAXV>(buf, M_blue, tw, fft_max, [&](int q) -> C2<T> {
        return q < L ? cmul(src(q), ldc(chirp, q)) : C2<T>{T(0), T(0)};
    });
    fft_lds<T, NT, MAXV>(buf, M_blue, tw, fft_max,
                         [&](int q) -> C2<T> { return cconj(cmul(buf[lpad(q)], ldc(chirpfft, q))); });
    return {buf, chirp, T(1) / T(M_blue)};
}

// ---------------------------------------------------------------------------
// S1: forward ring transform
// ---------------------------------------------------------------------------

// Workgroup -> (map, ring pair).  Consecutive workgroups are dealt to the 8
// XCDs in turn, so ring pairs are assigned to XCDs (h mod 8) and, within an
// XCD, all maps of one ring pair run back to back: their writes (reads) of
// the same Dsym rows then meet in that XCD's L2.
// `id` is the workgroup's index among the nmaps * npairs items of its group
// (a multiple of 8 away from its launch index, so id mod 8 is its XCD).
//   order 0 (default): ring pair h on XCD h mod 8, the maps of a pair back to
//     back there (their writes of one Dsym row meet in that XCD's L2);
//   order 1: pairs in order, the maps of a pair back to back, no XCD placement;
//   order 2: maps in order, all pairs of a map back to back.
__device__ __forceinline__ void ring_block_id(int id, int nmaps, int npairs, int& map, int& h, int order = 0) {
    if (order == 1) {
        map = id % nmaps;
        h = id / nmaps + 1;
        return;
    }
    if (order == 2) {
        map = id / npairs;
        h = id % npairs + 1;
        return;
    }
    if ((npairs & 7) == 0) {
        const int x = id & 7, s = id >> 3;
        h = (s / nmaps) * 8 + x + 1;
        map = s % nmaps;
    } else {
        map = id % nmaps;
        h = id / nmaps + 1;
    }
}
// The same for a launch of one group over an (nmaps, npairs) grid.
__device__ __forceinline__ void ring_block(int nmaps, int npairs, int& map, int& h) {
    ring_block_id(blockIdx.x + gridDim.x * blockIdx.y, nmaps, npairs, map, h);
}

// ---------------------------------------------------------------------------
// Work lists over the nside groups of a plan
// ---------------------------------------------------------------------------

// Group (index into the plan's GroupDesc array) and item index within it of
// work item `id` of a launch; false for a padding item.
// Both are workgroup-uniform; readfirstlane makes that explicit, so that
// the descriptor fields read through them stay in scalar registers.
__device__ __forceinline__ bool locate_item(const GroupRange& gr, int id, int& gi, int& local) {
    int i = 0;
    while (i + 1 < gr.n && i + 1 < kMaxGroups && id >= gr.start[i + 1]) ++i;
    i = __builtin_amdgcn_readfirstlane(i);
    gi = gr.first + i;
    local = __builtin_amdgcn_readfirstlane(id - gr.start[i]);
    return local < gr.count[i];
}

// The four blocks of one workspace region of a group, read like a Blocks4
// (R.p[b]): the block offsets stay in the group's descriptor in device
// memory, so a block picked by a run-time index (the parity of a mode) is one
// address computation and not a per-lane copy of a pointer array (copies of
// dynamically indexed structs would live in scratch memory).
template <class T>
struct RegionBlocks {
    struct Ptrs {
        char* ws;
        const int64_t* off;   // G.reg[r], null for an absent region
        __device__ __forceinline__ T* operator[](int b) const {
            return off ? reinterpret_cast<T*>(ws + off[b]) : nullptr;
        }
    } p;
};
template <class T>
__device__ __forceinline__ RegionBlocks<T> region_blocks(char* ws, const GroupDesc& G, int reg) {
    return RegionBlocks<T>{{ws, G.reg[reg]}};
}

// A workgroup-uniform value read from a descriptor, moved to scalar
// registers word by word (readfirstlane), so that it does not occupy vector
// registers for the rest of the kernel.
template <class V>
__device__ __forceinline__ V uniform(V v) {
    static_assert(sizeof(V) % 4 == 0, "32-bit words");
    uint32_t w[sizeof(V) / 4];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (unsigned i = 0; i < sizeof(V) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    V out;
    __builtin_memcpy(&out, w, sizeof(V));
    return out;
}

// The four block pointers of one region as scalars: at(i) picks one by
// selects, so a per-lane block index needs no indexable (scratch) copy.
template <class T>
struct Quad {
    T *b0, *b1, *b2, *b3;
    __device__ __forceinline__ T* at(int i) const { return i == 0 ? b0 : (i == 1 ? b1 : (i == 2 ? b2 : b3)); }
    __device__ __forceinline__ bool null() const { return b0 == nullptr; }
};
template <class T>
__device__ __forceinline__ Quad<T> region_quad(char* ws, const GroupDesc& G, int reg) {
    if (reg < 0) return Quad<T>{nullptr, nullptr, nullptr, nullptr};
    return Quad<T>{reinterpret_cast<T*>(ws + uniform(G.reg[reg][0])), reinterpret_cast<T*>(ws + uniform(G.reg[reg][1])),
                   reinterpret_cast<T*>(ws + uniform(G.reg[reg][2])), reinterpret_cast<T*>(ws + uniform(G.reg[reg][3]))};
}

// What the ring transform of one group writes to: the group's shape and the
// four blocks of its output region, as plain scalars.
template <class T>
struct RingOut {
    int nmaps, nside, p;
    int64_t N0, N1, cm0, cm1, ck0, ck1;
    T *d0, *d1, *d2, *d3;
};

// Item ranges of a launch: `count_of(desc)` items per group, each group's
// range starting at a multiple of 8.
template <class F>
static hipError_t make_range(const GroupLaunch& gl, F count_of, GroupRange& r) {
    if (gl.n < 0 || gl.n > kMaxGroups) return hipErrorInvalidValue;
    r = GroupRange{};
    r.first = gl.first;
    r.n = gl.n;
    int64_t at = 0;
    for (int i = 0; i < gl.n; ++i) {
        const int64_t c = count_of(gl.host[gl.first + i]);
        r.start[i] = int32_t(at);
        r.count[i] = int32_t(c);
        at += (c + 7) / 8 * 8;
        if (at >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    }
    r.start[gl.n] = int32_t(at);
    return hipSuccess;
}

// Grid of a launch over the range: one workgroup per item, or the persistent
// grid when it is smaller (a multiple of 8: the XCD of an item stays its
// index mod 8).
static unsigned list_grid(const GroupLaunch& gl, const GroupRange& r, bool persistent_ok) {
    const int total = r.start[r.n];
    if (persistent_ok && gl.grid_cap > 0 && gl.grid_cap < total) return unsigned(gl.grid_cap / 8 * 8);
    return unsigned(total);
}

// Ring kernels run NT = fft_max / 16 threads (256 up to nside 1024, 512 at
// nside 2048), so that every FFT of up to fft_max points keeps at most 16
// complex values per thread.  The forward transform can also run 512
// threads up to nside 1024 with at most MAXV = 8 values per thread (radix-8
// passes: one more pass, half the registers per thread, twice the waves).
constexpr int kRingMaxV = 16;
// Output modes k <= p per thread: ceil((2 nside + 1) / NT) with
// NT MAXV = 4 nside at the largest nside of each kernel.
constexpr int ring_kpt(int maxv) { return maxv / 2 + 1; }
constexpr int kRingKPT = ring_kpt(kRingMaxV);


// D_k, k <= p, of one ring from the half-length DFT R of its points (Step 1):
// the real DFT X_k = E_k + e^{-2 pi i k / n} O_k from the transform of
// z_q = x_{2q} + i x_{2q+1}, shifted to lambda = 0 on a shifted ring, scaled
// by 1/n; the Nyquist rule at k = n/2 (R3) and zero above.
template <class T>
__device__ __forceinline__ C2<T> ring_coeff(const DftOut<T>& R, int k, int n, bool shifted, int p, const T* roots) {
    const int L = n >> 1;
    const T invn = T(1) / T(n);
    C2<T> d = {T(0), T(0)};
    if (k <= p) {
        if (k < L) {
            const C2<T> zk = R.Z(k), zl = R.Z(k == 0 ? 0 : L - k);
            const C2<T> e = cscale(cadd(zk, cconj(zl)), T(0.5));
            const C2<T> dlt = csub(zk, cconj(zl));
            const C2<T> o = {T(0.5) * dlt.y, -T(0.5) * dlt.x};   // (zk - conj zl) / (2i)
            C2<T> X = cadd(e, cmul(ldc(roots, 2 * k), o));
            if (shifted) X = cmul(X, ldc(roots, k));
            d = cscale(X, invn);
        } else if (k == L) {
            const C2<T> z0 = R.Z(0);
            const T alpha = (z0.x - z0.y) * invn;
            if (L < p) d = {T(0), -T(0.5) * alpha};   // polar ring: alpha sin(L lambda)
            else d = {shifted ? T(0) : T(0.5) * alpha, T(0)};
        }
    }
    return d;
}

template <class T, int NT, int MAXV>
__device__ __forceinline__ void ring_spectrum(const double* x, int n, bool shifted, int p, FftTab<T> ft, C2<T>* buf,
                              C2<T> (&D)[ring_kpt(MAXV)]) {
    const int L = n >> 1, j = n >> 2;
    const int Mb = ft.chirpm[j];
    const T* chirp = ft.chirp + 2 * ft.chirpoff[j];
    const T* chirpfft = ft.chirpfft + 2 * ft.chirpfftoff[j];
    const T* roots = ft.roots + 2 * ft.rootoff[j];
    // z_q = x_{2q} + i x_{2q+1}: the real ring as L complex points
    auto src = [x](int q) -> C2<T> {
        const D2 v = *reinterpret_cast<const D2*>(x + 2 * q);
        return {T(v.x), T(v.y)};
    };
    const DftOut<T> R = ring_dft<T, NT, MAXV>(buf, L, Mb, chirp, chirpfft, ft.twiddle, ft.fft_max, src);
#pragma unroll
    for (int i = 0; i < ring_kpt(MAXV); ++i) D[i] = ring_coeff(R, threadIdx.x + i * NT, n, shifted, p, roots);
    // The next transform's first pass synchronises before it writes the buffer.
}

// LDS slots of one half of the ring kernels' buffer (a transform of up to
// fft_max / 2 points) and the whole buffer (one transform of fft_max points,
// or two halves side by side).
__host__ __device__ constexpr int ring_half_slots(int fft_max) { return fft_max / 2 + fft_max / 32 + 1; }
__host__ __device__ constexpr int ring_buffer_slots(int fft_max) {
    return (fft_max + fft_max / 16 + 1) > 2 * ring_half_slots(fft_max) ? fft_max + fft_max / 16 + 1
                                                                         : 2 * ring_half_slots(fft_max);
}

// Work item `id` of one group: ring pair h of map b (ring_block_id).
template <class T, int NT, int MAXV>
__device__ __forceinline__ void ring_forward_item(const double* __restrict__ maps,
                                                  const int64_t* __restrict__ map_off, const RingTab rt,
                                                  const FftTab<T> ft, const RingOut<T> o, int id, C2<T>* buf,
                                                  int order) {
    int b, h;
    ring_block_id(id, o.nmaps, 2 * o.nside, b, h, order);
    const int ns = o.nside, p = o.p;
    const double* m = maps + map_off[b];
    const bool equator = (h == 2 * ns);
    // Row starts and column steps of the two k parities (workgroup-uniform);
    // each lane picks its parity by a select.
    T* const bp0 = o.d0 + int64_t(h) * o.N0 + int64_t(b) * o.cm0;
    T* const bm0 = o.d1 + int64_t(h) * o.N0 + int64_t(b) * o.cm0;
    T* const bp1 = o.d2 + int64_t(h) * o.N1 + int64_t(b) * o.cm1;
    T* const bm1 = o.d3 + int64_t(h) * o.N1 + int64_t(b) * o.cm1;
    const int64_t ck0 = o.ck0, ck1 = o.ck1;
    auto store = [&](int k, C2<T> dp, C2<T> dm) {
        const bool odd = (k & 1) != 0;
        const int64_t col = int64_t(k >> 1) * (odd ? ck1 : ck0);
        T* bp = (odd ? bp1 : bp0) + col;
        T* bm = (odd ? bm1 : bm0) + col;
        bp[0] = dp.x;
        bp[1] = dp.y;
        bm[0] = dm.x;
        bm[1] = dm.y;
    };
    {
        // Both rings of a pair have n points and the same shift.  When their
        // transforms fit in half the buffer (every ring but the large
        // Bluestein ones and the equator), the two halves of the workgroup
        // transform them side by side.
        const int n = rt.n[h - 1], j = n >> 2, L = n >> 1;
        const int Mfft = ft.chirpm[j] ? ft.chirpm[j] : L;
        if (!equator && Mfft <= (ft.fft_max >> 1)) {
            constexpr int NH = NT / 2;
            const int half = threadIdx.x / NH;   // 0: ring h (north), 1: ring 4 nside - h
            const int r0 = half ? 4 * ns - h - 1 : h - 1;
            const bool shifted = rt.shifted[h - 1] != 0;
            const double* x = m + rt.start[r0];
            const T* chirp = ft.chirp + 2 * ft.chirpoff[j];
            const T* chirpfft = ft.chirpfft + 2 * ft.chirpfftoff[j];
            const T* roots = ft.roots + 2 * ft.rootoff[j];
            auto src = [x](int q) -> C2<T> {
                const D2 v = *reinterpret_cast<const D2*>(x + 2 * q);
                return {T(v.x), T(v.y)};
            };
            const int hs = ring_half_slots(ft.fft_max);
            DftOut<T> R = ring_dft<T, NH, MAXV>(buf + half * hs, L, ft.chirpm[j], chirp, chirpfft, ft.twiddle,
                                                ft.fft_max, src);
            __syncthreads();   // both spectra are in LDS
            DftOut<T> RN = R, RS = R;
            RN.buf = buf;
            RS.buf = buf + hs;
#pragma unroll
            for (int i = 0; i < ring_kpt(MAXV); ++i) {
                const int k = threadIdx.x + i * NT;
                if (k > p) continue;
                const C2<T> dn = ring_coeff(RN, k, n, shifted, p, roots);
                const C2<T> ds = ring_coeff(RS, k, n, shifted, p, roots);
                store(k, cscale(cadd(dn, ds), T(0.5)), cscale(csub(dn, ds), T(0.5)));
            }
            return;
        }
    }
    C2<T> DN[ring_kpt(MAXV)], DS[ring_kpt(MAXV)];
    {
        const int r0 = h - 1;
        ring_spectrum<T, NT, MAXV>(m + rt.start[r0], rt.n[r0], rt.shifted[r0] != 0, p, ft, buf, DN);
    }
    if (!equator) {
        const int r0 = 4 * ns - h - 1;
        ring_spectrum<T, NT, MAXV>(m + rt.start[r0], rt.n[r0], rt.shifted[r0] != 0, p, ft, buf, DS);
    }
#pragma unroll
    for (int i = 0; i < ring_kpt(MAXV); ++i) {
        const int k = threadIdx.x + i * NT;
        if (k > p) continue;
        if (equator) store(k, DN[i], C2<T>{T(0), T(0)});
        else store(k, cscale(cadd(DN[i], DS[i]), T(0.5)), cscale(csub(DN[i], DS[i]), T(0.5)));
    }
}

// S1 over the work list of every group of the launch (FP64 ring
// coefficients into region `reg`), one workgroup per item, or (PERSIST) a
// grid that walks the list; there the barrier at the end of an item keeps
// the next item's first LDS writes behind this item's last LDS reads.  The
// loop costs registers (256 VGPRs against 192, one wave per SIMD instead of
// two), so the persistent form is a candidate the autotuner measures.
template <int NT, int MAXV>
__device__ __forceinline__ void ring_forward_list_item(const double* __restrict__ maps,
                                                       const GroupDesc* __restrict__ gd, const GroupRange& gr,
                                                       char* ws, int reg, int id, C2<double>* buf, int order) {
    int gi, local;
    if (!locate_item(gr, id, gi, local)) return;
    const GroupDesc& G = gd[gi];
    const GroupDims& g = G.g;
    RingOut<double> o;
    o.nmaps = uniform(g.nmaps);
    o.nside = uniform(g.nside);
    o.p = uniform(g.p);
    o.N0 = uniform(g.N[0]);
    o.N1 = uniform(g.N[1]);
    o.cm0 = uniform(g.cm[0]);
    o.cm1 = uniform(g.cm[1]);
    o.ck0 = uniform(g.ck[0]);
    o.ck1 = uniform(g.ck[1]);
    o.d0 = reinterpret_cast<double*>(ws + uniform(G.reg[reg][0]));
    o.d1 = reinterpret_cast<double*>(ws + uniform(G.reg[reg][1]));
    o.d2 = reinterpret_cast<double*>(ws + uniform(G.reg[reg][2]));
    o.d3 = reinterpret_cast<double*>(ws + uniform(G.reg[reg][3]));
    ring_forward_item<double, NT, MAXV>(maps, uniform(G.map_off), uniform(G.rt), uniform(G.ft), o, local, buf, order);
}

// S1 over the work list of every group of the launch (FP64 ring
// coefficients into region `reg`), one workgroup per item.  (A persistent
// form that walks the list does not fit: its loop keeps more values live
// than the 256 VGPRs of a wave and spills to scratch memory, against 188
// VGPRs and no scratch for one item per workgroup.)
template <int NT, int MAXV>
__global__ __launch_bounds__(NT) void k_ring_forward(const double* __restrict__ maps,
                                                     const GroupDesc* __restrict__ gd, GroupRange gr, char* ws,
                                                     int reg, int order) {
    extern __shared__ unsigned char smem_raw[];
    C2<double>* buf = reinterpret_cast<C2<double>*>(smem_raw);
    ring_forward_list_item<NT, MAXV>(maps, gd, gr, ws, reg, blockIdx.x, buf, order);
}

// ---------------------------------------------------------------------------
// Equal-weight analysis, eq. (healsph): per-ring longitude sums
// ---------------------------------------------------------------------------

// F(m) = sum_q x_q e^{-i m lambda_q}, lambda_q = phi0 + 2 pi q / n, for the
// modes m = threadIdx.x + i NT <= p of one ring.  With the DFT of the real
// ring, X_t = sum_q x_q e^{-2 pi i q t / n} (X_{n-t} = conj X_t),
// F(m) = e^{-i m phi0} X_{m mod n}: unlike the interpolation of Step 1, modes
// at and beyond the ring's Nyquist mode n/2 repeat its spectrum (the sum over
// the ring's points aliases them), which is what the adjoint of the synthesis
// needs.
template <int NT>
__device__ __forceinline__ void ring_longitude_sums(const double* x, int n, bool shifted, int p, FftTab<double> ft,
                                                    C2<double>* buf, C2<double> (&F)[kRingKPT]) {
    const int L = n >> 1, j = n >> 2;
    const int Mb = ft.chirpm[j];
    const double* chirp = ft.chirp + 2 * ft.chirpoff[j];
    const double* chirpfft = ft.chirpfft + 2 * ft.chirpfftoff[j];
    const double* roots = ft.roots + 2 * ft.rootoff[j];   // e^{-i pi k / n}, k = 0..n
    auto src = [x](int q) -> C2<double> {
        const D2 v = *reinterpret_cast<const D2*>(x + 2 * q);
        return {v.x, v.y};
    };
    const DftOut<double> R = ring_dft<double, NT, kRingMaxV>(buf, L, Mb, chirp, chirpfft, ft.twiddle, ft.fft_max, src);
#pragma unroll
    for (int i = 0; i < kRingKPT; ++i) {
        const int m = threadIdx.x + i * NT;
        C2<double> X = {0.0, 0.0};
        if (m <= p) {
            int t = m % n;
            const bool upper = t > L;   // X_t = conj X_{n-t}
            if (upper) t = n - t;
            if (t == L) {
                const C2<double> z0 = R.Z(0);
                X = {z0.x - z0.y, 0.0};   // sum_q x_q (-1)^q
            } else {
                // X_t = E_t + e^{-2 pi i t / n} O_t from the L-point DFT of
                // z_q = x_{2q} + i x_{2q+1}
                const C2<double> zk = R.Z(t), zl = R.Z(t == 0 ? 0 : L - t);
                const C2<double> e = cscale(cadd(zk, cconj(zl)), 0.5);
                const C2<double> dlt = csub(zk, cconj(zl));
                const C2<double> o = {0.5 * dlt.y, -0.5 * dlt.x};
                X = cadd(e, cmul(ldc(roots, 2 * t), o));
            }
            if (upper) X = cconj(X);
            if (shifted) {
                // e^{-i pi m / n}, m mod 2n: the table holds k = 0..n
                const int u = m % (2 * n);
                const C2<double> ph = u <= n ? ldc(roots, u) : cscale(ldc(roots, u - n), -1.0);
                X = cmul(X, ph);
            }
        }
        F[i] = X;
    }
    // The next transform's first pass synchronises before it writes the buffer.
}

// Rows h = 1 .. 2 nside of Dsym for the equal-weight analysis: with the
// longitude sums F_N, F_S of the ring pair h, writes
//   W+ = scale (F_N + F_S),  W- = scale (F_N - F_S)
// (equator: W+ = scale F_N, W- = 0), scale = 4 pi / (12 nside^2), for every
// mode m = 0..p.  Since Pt_l^m(-z) = (-1)^{l+m} Pt_l^m(z), the order-m
// evaluation table of the synthesis, transposed, maps W to a_l^m.
template <int NT>
__global__ __launch_bounds__(NT) void k_ring_adjoint(const double* __restrict__ maps,
                                                     const int64_t* __restrict__ map_off, RingTab rt,
                                                     FftTab<double> ft, Blocks4<double> W, GroupDims g,
                                                     double scale) {
    extern __shared__ unsigned char smem_raw[];
    C2<double>* buf = reinterpret_cast<C2<double>*>(smem_raw);
    int b, h;
    ring_block(g.nmaps, 2 * g.nside, b, h);
    const int ns = g.nside, p = g.p;
    const double* m = maps + map_off[b];
    C2<double> FN[kRingKPT], FS[kRingKPT];
    {
        const int r0 = h - 1;
        ring_longitude_sums<NT>(m + rt.start[r0], rt.n[r0], rt.shifted[r0] != 0, p, ft, buf, FN);
    }
    const bool equator = (h == 2 * ns);
    if (!equator) {
        const int r0 = 4 * ns - h - 1;
        ring_longitude_sums<NT>(m + rt.start[r0], rt.n[r0], rt.shifted[r0] != 0, p, ft, buf, FS);
    }
#pragma unroll
    for (int i = 0; i < kRingKPT; ++i) {
        const int k = threadIdx.x + i * NT;
        if (k > p) continue;
        C2<double> wp, wm;
        if (equator) {
            wp = cscale(FN[i], scale);
            wm = {0.0, 0.0};
        } else {
            wp = cscale(cadd(FN[i], FS[i]), scale);
            wm = cscale(csub(FN[i], FS[i]), scale);
        }
        const int kpar = k & 1, kk = k >> 1;
        const int64_t col = int64_t(b) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
        const int64_t row = int64_t(h) * g.N[kpar];
        double* bp = W.p[2 * kpar + 0];
        double* bm = W.p[2 * kpar + 1];
        bp[row + col] = wp.x;
        bp[row + col + 1] = wp.y;
        bm[row + col] = wm.x;
        bm[row + col + 1] = wm.y;
    }
}

static size_t lds_slots_bytes(int slots, size_t elem) { return size_t(slots + slots / 16 + 1) * elem; }

static size_t ring_lds_bytes(int fft_max, size_t elem) {
    return size_t(ring_buffer_slots(std::max(fft_max, 256))) * elem;
}

hipError_t launch_ring_forward(const double* maps, const GroupLaunch& gl, int reg, hipStream_t s) {
    GroupRange r;
    if (hipError_t e = make_range(gl, [](const GroupDesc& G) { return int64_t(G.g.nmaps) * 2 * G.g.nside; }, r);
        e != hipSuccess)
        return e;
    if (r.start[r.n] == 0) return hipSuccess;
    int fmax = 0;
    for (int i = 0; i < gl.n; ++i) fmax = std::max(fmax, gl.host[gl.first + i].ft.fft_max);
    const size_t shm = ring_lds_bytes(fmax, sizeof(C2<double>));
    const dim3 grid(list_grid(gl, r, false));
    const int order = gl.variant >= 0 && gl.variant <= 2 ? gl.variant : 0;
    if (ring_threads(fmax) == 512)
        hipLaunchKernelGGL((k_ring_forward<512, 16>), grid, dim3(512), shm, s, maps, gl.dev, r, gl.ws, reg, order);
    else if (gl.threads == 512)
        hipLaunchKernelGGL((k_ring_forward<512, 8>), grid, dim3(512), shm, s, maps, gl.dev, r, gl.ws, reg, order);
    else
        hipLaunchKernelGGL((k_ring_forward<256, 16>), grid, dim3(256), shm, s, maps, gl.dev, r, gl.ws, reg, order);
    return hipGetLastError();
}

hipError_t launch_ring_adjoint(const double* maps, const int64_t* map_off, RingTab rt, FftTab<double> ft,
                               Blocks4<double> W, const GroupDims& g, double scale, hipStream_t s) {
    dim3 grid(g.nmaps, 2 * g.nside);
    const size_t shm = ring_lds_bytes(ft.fft_max, sizeof(C2<double>));
    if (ring_threads(ft.fft_max) == 256)
        hipLaunchKernelGGL(k_ring_adjoint<256>, grid, dim3(256), shm, s, maps, map_off, rt, ft, W, g, scale);
    else
        hipLaunchKernelGGL(k_ring_adjoint<512>, grid, dim3(512), shm, s, maps, map_off, rt, ft, W, g, scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// S2: pole row
// ---------------------------------------------------------------------------

template <class T, class BK>
__device__ __forceinline__ void pole_item(BK D, const GroupDims& g, double w0, double w1, double w2, int64_t i) {
    const int64_t N0 = g.N[0], N1 = g.N[1];
    const int64_t total = 2 * N0 + 2 * N1;
    if (i >= total) return;
    int blk;
    int64_t col, N;
    if (i < N0) { blk = 0; col = i; N = N0; }
    else if (i < 2 * N0) { blk = 1; col = i - N0; N = N0; }
    else if (i < 2 * N0 + N1) { blk = 2; col = i - 2 * N0; N = N1; }
    else { blk = 3; col = i - 2 * N0 - N1; N = N1; }
    T* P = D.p[blk];
    T val = T(0);
    // (k' = 0, real part) columns of the k-even blocks hold the pole value
    const bool k0re = g.modemajor ? (col < 2 * int64_t(g.nmaps) && (col & 1) == 0) : ((col % g.Npm[0]) == 0);
    if (blk < 2 && k0re) {
        // k = 0, real part: the pole value (f_N +- f_S) / 2 from the ring means
        val = T(w0 * double(P[1 * N + col]) + w1 * double(P[2 * N + col]) + w2 * double(P[3 * N + col]));
    }
    P[col] = val;
}

// Work item: 256 consecutive pole-row entries of one group.
template <class T>
__global__ __launch_bounds__(256) void k_pole(const GroupDesc* __restrict__ gd, GroupRange gr, char* ws, int reg) {
    int gi, local;
    if (!locate_item(gr, blockIdx.x, gi, local)) return;
    const GroupDesc& G = gd[gi];
    pole_item<T>(region_blocks<T>(ws, G, reg), G.g, G.pole_w[0], G.pole_w[1], G.pole_w[2],
                 int64_t(local) * 256 + threadIdx.x);
}

template <class T>
hipError_t launch_pole(const GroupLaunch& gl, int reg, hipStream_t s) {
    GroupRange r;
    if (hipError_t e = make_range(
            gl, [](const GroupDesc& G) { return (2 * G.g.N[0] + 2 * G.g.N[1] + 255) / 256; }, r);
        e != hipSuccess)
        return e;
    if (r.start[r.n] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pole<T>, dim3(list_grid(gl, r, false)), dim3(256), 0, s, gl.dev, r, gl.ws, reg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped GEMM on MFMA: C[m][n] = sum_k A[k][m] B[k][n]
// ---------------------------------------------------------------------------

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct MfmaAcc;
// Operand layout (both precisions, measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] of the 16x4 / 4x16 operands.
// Accumulator register r of lane l holds D[row][l % 16] with
// row = 4 r + l / 16 for f64_16x16x4 and row = 4 (l / 16) + r for f32_16x16x4.
template <>
struct MfmaAcc<double> {
    using V = v4d;
    static __device__ __forceinline__ V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct MfmaAcc<float> {
    using V = v4f;
    static __device__ __forceinline__ V mma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int GBM = kGemmBM, GBN = kGemmBN, GBK = kGemmBK;
// Row pad of the LDS tiles: a row stride of GBM + 16 elements puts the four
// k rows that one MFMA operand load touches on disjoint bank ranges.
constexpr int GPAD = 16;

// 16-byte vector of T (4 floats / 2 doubles), as written to LDS.
template <class T>
struct alignas(16) V16 {
    T v[16 / sizeof(T)];
};

typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
// native 16-byte vector of T and native (re, im) pair of T
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = v4f;
};
template <>
struct Vec16<double> {
    using type = v2d;
};
template <class T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = v2f;
};
template <>
struct Vec2<double> {
    using type = v2d;
};

// Raw buffer descriptors (gfx9 family): word 3 selects 32-bit data with no
// swizzle, and a byte offset at or past the descriptor's record count reads
// as zero.  kGemmOOB is past every descriptor the GEMM builds (records stay
// below 2^31, checked when a problem list is built).
constexpr int kBufferWord3 = 0x00020000;

// sizeof(V) bytes (4, 8 or 16) at byte offset `off` of the buffer
template <class V>
__device__ __forceinline__ V buffer_load(__amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(V) == 16) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    else if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// C[m][n] = sum_k A[k][m] B[k][n] for a list of problems; one 128 x 128 tile
// of one problem per workgroup (4 waves of 64 x 64 each), k in steps of 16
// through double-buffered LDS tiles, global loads issued ahead of use.  B and C columns come in (re, im)
// pairs: column n lives at (n >> 1) * pair_stride + (n & 1).  A wave skips
// the MFMAs of its 16-row blocks past the problem's last row and of its
// 16-column blocks past the last column (NI, NJ = live row / column blocks of
// the wave, template arguments so that the block loops stay unrolled; a
// column tile that holds only the last few columns of a problem -- N = 146
// for 73 maps -- then costs a fraction of a full tile).
template <class T, class TB, int NI, int NJ>
__device__ __forceinline__ void gemm_tile(const GemmProblem<T>& P, int m0, int n0, const TB* __restrict__ B,
                                          T* __restrict__ C, T (*As)[GBK][GBM + GPAD],
                                          T (*Bs)[GBK][GBN + GPAD]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    using Acc = MfmaAcc<T>;
    typename Acc::V acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = typename Acc::V{0, 0, 0, 0};

    // Each thread stages 8 elements of one k row of each tile: 16-byte vector
    // q of the thread sits at column 16 VE q + VE (tid % 16), so the 16 lanes
    // of a row write one contiguous 256-byte run per store (every LDS bank
    // once) and read contiguous 256-byte runs from memory.
    // The staging loads are buffer loads: per k step one descriptor for A and
    // one for B cover the step's rows that lie inside the problem (records =
    // rows x row bytes), and an element outside the problem's columns gets an
    // offset past every descriptor.  The hardware returns zero for both, so
    // no loaded register is touched before the LDS store (B stays in its
    // storage type until then) and the loads of a step stay in flight behind
    // the MFMAs of the steps before it.
    // The offsets and descriptor sizes come from GemmStage / gemm_*_offset
    // (kernels.h), which the host-side replay of the problem lists also runs.
    constexpr int VE = GemmStage<T>::VE;
    const int lr = GemmStage<T>::row(tid);   // 0..15
    auto ecol = [&](int e) { return GemmStage<T>::col(tid, e); };
    const bool avec = gemm_a_vector(P);
    using VT = typename Vec16<T>::type;
    using PT = typename Vec2<TB>::type;
    auto gload = [&](int k0, T (&ra)[8], TB (&rb)[8]) {
        const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<T*>(P.A + int64_t(k0) * P.lda), 0, int(gemm_a_records(P, k0)), kBufferWord3);
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<TB*>(B + int64_t(k0) * P.ldb), 0, int(gemm_b_records<T, TB>(P, k0)), kBufferWord3);
        if (avec) {
#pragma unroll
            for (int e = 0; e < 8; e += VE) {
                const VT v = buffer_load<VT>(rA, int(gemm_a_offset(P, true, m0, tid, e)));
#pragma unroll
                for (int q = 0; q < VE; ++q) ra[e + q] = v[q];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) ra[e] = buffer_load<T>(rA, int(gemm_a_offset(P, false, m0, tid, e)));
        }
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const PT v = buffer_load<PT>(rB, int(gemm_b_offset<T, TB>(P, n0, tid, e)));
            rb[e] = v[0];
            rb[e + 1] = v[1];
        }
    };
    auto lstore = [&](int buf, const T (&ra)[8], const TB (&rb)[8]) {
#pragma unroll
        for (int e = 0; e < 8; e += VE) {
            V16<T> va, vb;
#pragma unroll
            for (int q = 0; q < VE; ++q) {
                va.v[q] = ra[e + q];
                vb.v[q] = T(rb[e + q]);
            }
            *reinterpret_cast<V16<T>*>(&As[buf][lr][ecol(e)]) = va;
            *reinterpret_cast<V16<T>*>(&Bs[buf][lr][ecol(e)]) = vb;
        }
    };
    auto compute = [&](int cur) {
        if constexpr (NI > 0) {
#pragma unroll
            for (int kk = 0; kk < GBK / 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                T a[NI], b[NJ];
#pragma unroll
                for (int i = 0; i < NI; ++i) a[i] = As[cur][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < NJ; ++j) b[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) acc[i][j] = Acc::mma(a[i], b[j], acc[i][j]);
            }
        }
    };
    // Step s of 16 k rows lives in LDS buffer s & 1 and is staged through
    // register set s & 1, its global loads issued two steps ahead.
    const int nk = (P.K + GBK - 1) / GBK;
    T ra0[8], ra1[8];
    TB rb0[8], rb1[8];
    gload(0, ra0, rb0);
    lstore(0, ra0, rb0);
    if (nk > 1) gload(GBK, ra1, rb1);
    if (nk > 2) gload(2 * GBK, ra0, rb0);
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
        compute(0);
        lstore(1, ra1, rb1);
        if (kt + 3 < nk) gload((kt + 3) * GBK, ra1, rb1);
        __syncthreads();
        compute(1);
        if (kt + 2 < nk) lstore(0, ra0, rb0);
        if (kt + 4 < nk) gload((kt + 4) * GBK, ra0, rb0);
        __syncthreads();
    }
    if (kt < nk) compute(0);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int nn = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mm = m0 + wm * 64 + i * 16 + Acc::row(lane, r);
                if (mm < P.M && nn < P.N)
                    C[int64_t(mm) * P.ldc + int64_t(nn >> 1) * P.cps + (nn & 1)] = acc[i][j][r];
            }
        }
    }
}

// Live 16-wide blocks of a wave's 64 rows (columns) when `left` rows
// (columns) of the problem remain from the wave's first one: 0..4.
__device__ __forceinline__ int gemm_live_blocks(int left) {
    return left <= 0 ? 0 : (left >= 64 ? 4 : (left + 15) / 16);
}

// TB: storage type of B (FP64 B is rounded to T as it is staged).
template <class T, class TB>
__global__ __launch_bounds__(256, sizeof(T) == 8 || sizeof(TB) == 8 ? 2 : 3) void k_gemm(const GemmProblem<T>* __restrict__ probs,
                                              const int32_t* __restrict__ tmap, const TB* __restrict__ Bbase,
                                              T* __restrict__ Cbase) {
    __shared__ T As[2][GBK][GBM + GPAD];
    __shared__ T Bs[2][GBK][GBN + GPAD];
    const int pi = tmap[2 * blockIdx.x];
    if (pi < 0) return;
    const GemmProblem<T> P = probs[pi];
    const int tile = tmap[2 * blockIdx.x + 1];
    const int tm = tile / P.tiles_n, tn = tile % P.tiles_n;
    const int m0 = tm * GBM, n0 = tn * GBN;
    const TB* B = Bbase + P.boff;
    T* C = Cbase + P.coff;
    // live 16-row and 16-column blocks of this wave's 64 x 64 (wave-uniform);
    // three live column blocks run as four (the fourth multiplies the zeros
    // the out-of-range B loads stage, and its stores are masked)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ni = gemm_live_blocks(P.M - m0 - (wave >> 1) * 64);
    int nj = gemm_live_blocks(P.N - n0 - (wave & 1) * 64);
    if (nj == 3) nj = 4;
    if (ni == 0 || nj == 0) {
        gemm_tile<T, TB, 0, 4>(P, m0, n0, B, C, As, Bs);
        return;
    }
    switch (nj * 8 + ni) {
        case 4 * 8 + 4: gemm_tile<T, TB, 4, 4>(P, m0, n0, B, C, As, Bs); break;
        case 4 * 8 + 3: gemm_tile<T, TB, 3, 4>(P, m0, n0, B, C, As, Bs); break;
        case 4 * 8 + 2: gemm_tile<T, TB, 2, 4>(P, m0, n0, B, C, As, Bs); break;
        case 4 * 8 + 1: gemm_tile<T, TB, 1, 4>(P, m0, n0, B, C, As, Bs); break;
        case 2 * 8 + 4: gemm_tile<T, TB, 4, 2>(P, m0, n0, B, C, As, Bs); break;
        case 2 * 8 + 3: gemm_tile<T, TB, 3, 2>(P, m0, n0, B, C, As, Bs); break;
        case 2 * 8 + 2: gemm_tile<T, TB, 2, 2>(P, m0, n0, B, C, As, Bs); break;
        case 2 * 8 + 1: gemm_tile<T, TB, 1, 2>(P, m0, n0, B, C, As, Bs); break;
        case 1 * 8 + 4: gemm_tile<T, TB, 4, 1>(P, m0, n0, B, C, As, Bs); break;
        case 1 * 8 + 3: gemm_tile<T, TB, 3, 1>(P, m0, n0, B, C, As, Bs); break;
        case 1 * 8 + 2: gemm_tile<T, TB, 2, 1>(P, m0, n0, B, C, As, Bs); break;
        default: gemm_tile<T, TB, 1, 1>(P, m0, n0, B, C, As, Bs); break;
    }
}

template <class T>
int finalize_gemm_problems(GemmProblem<T>* p, int n) {
    int t = 0;
    for (int i = 0; i < n; ++i) {
        const int tm = (p[i].M + GBM - 1) / GBM;
        p[i].tiles_n = (p[i].N + GBN - 1) / GBN;
        p[i].tile_begin = t;
        t += tm * p[i].tiles_n;
    }
    return t;
}

template <class T>
std::vector<int32_t> xcd_tile_map(const GemmProblem<T>* p, int n) {
    constexpr int kXcd = 8;
    std::vector<std::vector<int32_t>> per(kXcd);
    for (int i = 0; i < n; ++i) {
        const int tiles = ((p[i].M + GBM - 1) / GBM) * p[i].tiles_n;
        for (int t = 0; t < tiles; ++t) {
            per[i % kXcd].push_back(i);
            per[i % kXcd].push_back(t);
        }
    }
    size_t len = 0;
    for (auto& v : per) len = std::max(len, v.size() / 2);
    std::vector<int32_t> out(2 * len * kXcd, -1);
    for (int x = 0; x < kXcd; ++x)
        for (size_t s = 0; s < per[x].size() / 2; ++s) {
            out[2 * (s * kXcd + x)] = per[x][2 * s];
            out[2 * (s * kXcd + x) + 1] = per[x][2 * s + 1];
        }
    return out;
}

template <class T, class TB>
hipError_t launch_gemm(const GemmProblem<T>* probs_dev, const int32_t* tmap_dev, int nslots, const TB* Bbase,
                       T* Cbase, hipStream_t s) {
    if (nslots == 0) return hipSuccess;
    hipLaunchKernelGGL((k_gemm<T, TB>), dim3(nslots), dim3(256), 0, s, probs_dev, tmap_dev, Bbase, Cbase);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Set-up helpers for the per-order tables
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_replicate(const T* __restrict__ mat, int64_t rs, int64_t cs, int nl, int h_first, int h_last,
                            T* __restrict__ Uv, int nk, int nv) {
    // one thread per (l', v, k', c)
    const int64_t npm = 2 * int64_t(nk);
    const int64_t total = int64_t(nl) * nv * npm;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int lp = int(i / (nv * npm));
    const int64_t rem = i % (nv * npm);
    const int v = int(rem / npm);
    const int c = int(rem % 2);
    const int h = h_first + 2 * v + c;
    Uv[i] = (h <= h_last) ? mat[int64_t(h) * rs + int64_t(lp) * cs] : T(0);
}

template <class T>
hipError_t launch_replicate(const T* mat, int64_t rs, int64_t cs, int nl, int h_first, int h_last, T* Uv, int nk,
                            int nv, hipStream_t s) {
    const int64_t total = int64_t(nl) * nv * 2 * nk;
    hipLaunchKernelGGL(k_replicate<T>, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, mat, rs, cs, nl,
                       h_first, h_last, Uv, nk, nv);
    return hipGetLastError();
}

template <class T>
__global__ void k_scatter_tables(const T* __restrict__ Uv, int nl, int nk, int nv, int h_first, int h_last,
                                 const int64_t* __restrict__ off, const int32_t* __restrict__ h0v, int ldm_syn,
                                 int synthesis, T* __restrict__ tab) {
    const int64_t npm = 2 * int64_t(nk);
    const int64_t total = int64_t(nl) * nv * npm;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int lp = int(i / (nv * npm));
    const int64_t rem = i % (nv * npm);
    const int v = int(rem / npm);
    const int kk = int((rem % npm) >> 1);
    const int c = int(rem % 2);
    const int h = h_first + 2 * v + c;
    if (h > h_last || lp < kk) return;
    const int M = nl - kk;
    if (synthesis) {
        if (h < 1) return;
        tab[off[kk] + int64_t(lp - kk) * ldm_syn + (h - 1)] = Uv[i];
    } else {
        const int h0 = h0v[kk];
        if (h < h0) return;
        tab[off[kk] + int64_t(h - h0) * order_table_lda(M) + (lp - kk)] = Uv[i];
    }
}

template <class T>
hipError_t launch_scatter_tables(const T* Uv, int nl, int nk, int nv, int h_first, int h_last, const int64_t* off,
                                 const int32_t* h0, int ldm_syn, bool synthesis, T* tab, hipStream_t s) {
    const int64_t total = int64_t(nl) * nv * 2 * nk;
    hipLaunchKernelGGL(k_scatter_tables<T>, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, Uv, nl, nk, nv,
                       h_first, h_last, off, h0, ldm_syn, synthesis ? 1 : 0, tab);
    return hipGetLastError();
}

__global__ void k_convert(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = float(in[i]);
}

hipError_t launch_convert(const double* in, float* out, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

// adj[aoff[k']] [h][l] = syn[soff[k']] [l][h] for h < H, l < M = nl - k'
// (adjoint row stride order_table_lda(M)); one 32 x 32 tile through LDS per
// workgroup, blockIdx.y = k'.
__global__ __launch_bounds__(256) void k_transpose_orders(const double* __restrict__ syn,
                                                          const int64_t* __restrict__ soff,
                                                          double* __restrict__ adj,
                                                          const int64_t* __restrict__ aoff, int nl, int H) {
    __shared__ double tile[32][33];
    const int kk = blockIdx.y;
    const int M = nl - kk;
    const int tiles_h = (H + 31) / 32;
    const int th = blockIdx.x % tiles_h, tl = blockIdx.x / tiles_h;
    const int l0 = tl * 32, h0 = th * 32;
    if (l0 >= M) return;   // whole workgroup: no barrier is skipped by part of it
    const int lda = order_table_lda(M);
    const double* S = syn + soff[kk];
    double* A = adj + aoff[kk];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int l = l0 + r, h = h0 + tx;
        tile[r][tx] = (l < M && h < H) ? S[int64_t(l) * H + h] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int h = h0 + r, l = l0 + tx;
        if (h < H && l < M) A[int64_t(h) * lda + l] = tile[tx][r];
    }
}

hipError_t launch_transpose_orders(const double* syn, const int64_t* soff, double* adj, const int64_t* aoff, int nl,
                                   int nk, int H, hipStream_t s) {
    if (nk == 0 || nl == 0) return hipSuccess;
    dim3 grid(unsigned(((H + 31) / 32) * ((nl + 31) / 32)), unsigned(nk));
    hipLaunchKernelGGL(k_transpose_orders, grid, dim3(256), 0, s, syn, soff, adj, aoff, nl, H);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// S4: Givens sweeps.
//
// Column k' of block b needs sweeps t = 1 .. k' (order m' = 2t + kpar) in
// that order for analysis (each sweep: a carry runs up the chain l' = t-1 ..
// nl-1, rotating (carry, x[l']) and dropping the final carry), and t = k' ..
// 1 with the transposed rotations for synthesis (a zero carry runs down the
// chain and is deposited at l' = t-1).  The angles depend on (t, l') only,
// so they are the same for every map and every column that needs sweep t.
//
// One workgroup = SW_WAVES waves on the same 32 columns k' (lane = (k',
// re/im)) of MB maps of one block; each lane carries its column for all MB
// maps, so every angle pair read serves MB rotations per lane.  Sweeps are
// grouped in aligned blocks of SW (t = SW q + 1 .. SW q + SW); in one pass
// wave w applies block q0 + w, so a pass applies SW * SW_WAVES sweeps and
// streams the chains through HBM once.  Chain values move through the waves
// in chunks of SW_CHUNK positions: wave 0 reads from global memory (one
// chunk ahead), hands each chunk to wave 1 through LDS, .., the last wave
// writes back; at step s wave w works on chunk s - w, with a barrier per
// step (four positions per chunk: a quarter of a barrier per position, at
// 128 VGPRs for two maps per lane).  The carries of a wave's sweeps stay in
// registers for the pass; the angles come through the scalar cache, the SW
// pairs of a position in one batch.  Columns that need fewer sweeps than
// their neighbours are masked per lane only in the wave blocks that contain
// their last sweep.
// ---------------------------------------------------------------------------

constexpr int SW = 8;
constexpr int SW_WAVES = 8;
constexpr int SW_CHUNK = 4;
constexpr int kSweepCols = 32;

__device__ __forceinline__ void sweep_locate(const GroupDims& g, int nmg, int& blk, int& grp, int& mg) {
    // work items ordered longest first: highest column groups of all blocks first
    int w = blockIdx.x;
    mg = w % nmg;
    w /= nmg;
    int ng[4], gmax = 0;
    for (int b = 0; b < 4; ++b) {
        ng[b] = (g.nk[b] + kSweepCols - 1) / kSweepCols;
        gmax = max(gmax, ng[b]);
    }
    for (int r = gmax - 1; r >= 0; --r) {
        for (int b = 0; b < 4; ++b) {
            if (r < ng[b]) {
                if (w == 0) {
                    blk = b;
                    grp = r;
                    return;
                }
                --w;
            }
        }
    }
    blk = 0;
    grp = 0;
}

// The angle table is read-only while a sweep kernel runs: reading it through
// the constant address space lets wave-uniform loads use the scalar cache.
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ ConstPtr<T> as_const(const T* p) {
    return (ConstPtr<T>)(p);
}

// The SW angle pairs of sweeps tb .. tb+SW-1 at one position, loaded
// together (one batch of scalar loads and one wait, instead of a load and a
// wait in front of every rotation).  The row of the table holds tpad >= the
// next multiple of SW above the last sweep of any busy wave, so the whole
// block is in bounds even where its last sweeps are past the group's.
template <class T>
struct Angles {
    T c[SW], s[SW];
};

template <class T>
__device__ __forceinline__ Angles<T> load_angles(ConstPtr<T> cs) {
    Angles<T> a;
#pragma unroll
    for (int j = 0; j < SW; ++j) {
        a.c[j] = cs[2 * j];
        a.s[j] = cs[2 * j + 1];
    }
    return a;
}

// forward sweeps tb .. tb+SW-1 of one wave at position lp, for MB maps.
// Sweep t rotates at positions lp >= t and takes its carry at lp = t - 1, so
// at a given lp the wave applies the first nrot sweeps and then (if it is
// one of its own) starts the carry of sweep lp + 1.
// ALL: every sweep of the block rotates here and none starts (the interior
// of the chain), with no per-sweep branch.
template <class T, int MB, bool MASK, bool ALL>
__device__ __forceinline__ void fwd_rot(T (&v)[MB], int lp, int tb, int tg, int kk, T (&carry)[SW][MB],
                                        const Angles<T>& an) {
    const int nrot = ALL ? SW : max(0, min(min(lp - tb + 1, tg - tb + 1), SW));   // wave-uniform
    const int jinit = ALL ? -1 : (lp - tb + 1 < SW && lp + 1 <= tg) ? lp - tb + 1 : -1;
    T vf[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) vf[b] = v[b];
#pragma unroll
    for (int j = 0; j < SW; ++j) {
        if (j < nrot) {
            const int t = tb + j;
            const T c = an.c[j], s = an.s[j];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                // explicit fma order: every instantiation rounds identically
                const T nv = fma(c, carry[j][b], s * v[b]);
                carry[j][b] = fma(c, v[b], -(s * carry[j][b]));
                v[b] = nv;
                if (MASK) {
                    if (t <= kk) vf[b] = v[b];
                } else {
                    vf[b] = v[b];
                }
            }
        } else if (j == jinit) {
#pragma unroll
            for (int b = 0; b < MB; ++b) carry[j][b] = v[b];
        }
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) v[b] = vf[b];
}

template <class T, int MB, bool MASK>
__device__ __forceinline__ void fwd_position(T (&v)[MB], int lp, int tb, int tg, int kk, T (&carry)[SW][MB],
                                             const Angles<T>& an) {
    if (lp - tb + 1 >= SW && tg - tb + 1 >= SW) fwd_rot<T, MB, MASK, true>(v, lp, tb, tg, kk, carry, an);
    else fwd_rot<T, MB, MASK, false>(v, lp, tb, tg, kk, carry, an);
}

// backward (synthesis) sweeps tb+SW-1 down to tb at position lp, for MB maps
template <class T, int MB, bool MASK, bool ALL>
__device__ __forceinline__ void bwd_rot(T (&v)[MB], int lp, int tb, int tg, int kk, T (&carry)[SW][MB],
                                        const Angles<T>& an) {
#pragma unroll
    for (int jj = 0; jj < SW; ++jj) {
        const int j = SW - 1 - jj;
        const int t = tb + j;
        if (!ALL && t > tg) continue;
        const bool act = MASK ? (t <= kk) : true;
        if (ALL || lp >= t) {
            const T c = an.c[j], s = an.s[j];
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const T nv = fma(s, v[b], c * carry[j][b]);
                const T nc = fma(c, v[b], -(s * carry[j][b]));
                if (act) {
                    v[b] = nv;
                    carry[j][b] = nc;
                }
            }
        } else if (lp == t - 1) {
            if (act) {
#pragma unroll
                for (int b = 0; b < MB; ++b) v[b] = carry[j][b];
            }
        }
    }
}

template <class T, int MB, bool MASK>
__device__ __forceinline__ void bwd_position(T (&v)[MB], int lp, int tb, int tg, int kk, T (&carry)[SW][MB],
                                             const Angles<T>& an) {
    if (tb + SW - 1 <= tg && lp >= tb + SW - 1) bwd_rot<T, MB, MASK, true>(v, lp, tb, tg, kk, carry, an);
    else bwd_rot<T, MB, MASK, false>(v, lp, tb, tg, kk, carry, an);
}

template <class T, int MB, bool FWD>
__global__ __launch_bounds__(64 * SW_WAVES) void k_sweep(Blocks4<T> U, Blocks4<const T> G, GroupDims g) {
    __shared__ T slots[SW_WAVES][2][SW_CHUNK][MB][64];
    const int nmg = (g.nmaps + MB - 1) / MB;
    int blk, grp, mg;
    sweep_locate(g, nmg, blk, grp, mg);
    const int kpar = blk >> 1;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int lane = threadIdx.x & 63;
    const int kk = grp * kSweepCols + (lane >> 1);
    const int nk = g.nk[blk], nl = g.nl[blk], tpad = g.tpad[blk];
    const int64_t N = g.N[kpar];
    const bool kvalid = kk < nk;
    const int kcol = kvalid ? kk : nk - 1;
    T* col[MB];
    bool ok[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int map = mg * MB + b;
        ok[b] = kvalid && map < g.nmaps;
        col[b] = U.p[blk] + int64_t(map < g.nmaps ? map : 0) * g.Npm[kpar] + 2 * kcol + (lane & 1);
    }
    const T* Gt = G.p[blk];
    const int tg = min(grp * kSweepCols + kSweepCols - 1, nk - 1);
    const int kmin = grp * kSweepCols;
    const int qtop = (tg - 1) / SW;
    const int npass = qtop / SW_WAVES + 1;
    for (int pass = 0; pass < npass; ++pass) {
        // sweep block of this wave and the chain range of the pass
        int q, lo;
        if (FWD) {
            q = pass * SW_WAVES + wave;
            lo = pass * SW_WAVES * SW;                  // first position: t0 - 1
        } else {
            const int q0 = qtop - pass * SW_WAVES;
            q = q0 - wave;
            lo = max(q0 - SW_WAVES + 1, 0) * SW;        // lowest deposit position
        }
        const int tb = q * SW + 1;
        const bool busy = FWD ? (tb <= tg) : (q >= 0);
        const bool mask = busy && (tb + SW - 1 > kmin);
        T carry[SW][MB];
#pragma unroll
        for (int j = 0; j < SW; ++j)
#pragma unroll
            for (int b = 0; b < MB; ++b) carry[j][b] = T(0);
        const int npos = nl - lo;
        const int nchunks = (npos + SW_CHUNK - 1) / SW_CHUNK;
        // position of chunk element (c, i)
        auto posof = [&](int c, int i) { return FWD ? lo + c * SW_CHUNK + i : nl - 1 - (c * SW_CHUNK + i); };
        T nx[SW_CHUNK][MB];
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < SW_CHUNK; ++i) {
                const int lp = posof(0, i);
                const bool in = FWD ? (lp < nl) : (lp >= lo);
#pragma unroll
                for (int b = 0; b < MB; ++b) nx[i][b] = in ? col[b][int64_t(lp) * N] : T(0);
            }
        }
        for (int s = 0; s < nchunks + SW_WAVES - 1; ++s) {
            const int c = s - wave;
            if (c >= 0 && c < nchunks) {
                T v[SW_CHUNK][MB];
                if (wave == 0) {
#pragma unroll
                    for (int i = 0; i < SW_CHUNK; ++i)
#pragma unroll
                        for (int b = 0; b < MB; ++b) v[i][b] = nx[i][b];
                    if (c + 1 < nchunks) {
#pragma unroll
                        for (int i = 0; i < SW_CHUNK; ++i) {
                            const int lp = posof(c + 1, i);
                            const bool in = FWD ? (lp < nl) : (lp >= lo);
#pragma unroll
                            for (int b = 0; b < MB; ++b) nx[i][b] = in ? col[b][int64_t(lp) * N] : T(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < SW_CHUNK; ++i)
#pragma unroll
                        for (int b = 0; b < MB; ++b) v[i][b] = slots[wave][c & 1][i][b][lane];
                }
#pragma unroll
                for (int i = 0; i < SW_CHUNK; ++i) {
                    const int lp = posof(c, i);
                    const bool in = FWD ? (lp < nl) : (lp >= lo);
                    if (busy && in) {
                        const Angles<T> an = load_angles<T>(as_const(Gt + (int64_t(lp) * tpad + (tb - 1)) * 2));
                        if (FWD) {
                            if (mask) fwd_position<T, MB, true>(v[i], lp, tb, tg, kk, carry, an);
                            else fwd_position<T, MB, false>(v[i], lp, tb, tg, kk, carry, an);
                        } else {
                            if (mask) bwd_position<T, MB, true>(v[i], lp, tb, tg, kk, carry, an);
                            else bwd_position<T, MB, false>(v[i], lp, tb, tg, kk, carry, an);
                        }
                    }
                    if (wave == SW_WAVES - 1) {
                        if (in) {
#pragma unroll
                            for (int b = 0; b < MB; ++b)
                                if (ok[b]) col[b][int64_t(lp) * N] = v[i][b];
                        }
                    } else {
#pragma unroll
                        for (int b = 0; b < MB; ++b) slots[wave + 1][c & 1][i][b][lane] = v[i][b];
                    }
                }
            }
            __syncthreads();
        }
        __threadfence_block();
        __syncthreads();
    }
}

static int sweep_workgroups(const GroupDims& g, int mb) {
    int w = 0;
    for (int b = 0; b < 4; ++b) w += (g.nk[b] + kSweepCols - 1) / kSweepCols;
    return w * ((g.nmaps + mb - 1) / mb);
}

#ifndef HP2SPH_SWEEP_MB_MAX
#define HP2SPH_SWEEP_MB_MAX 2   // maps carried per lane by the sweep kernels (1, 2 or 4)
#endif

template <class T, bool FWD>
static hipError_t launch_sweep(Blocks4<T> U, Blocks4<const T> G, const GroupDims& g, hipStream_t s) {
    if (HP2SPH_SWEEP_MB_MAX >= 4 && g.nmaps >= 4) {
        hipLaunchKernelGGL((k_sweep<T, 4, FWD>), dim3(sweep_workgroups(g, 4)), dim3(64 * SW_WAVES), 0, s, U, G, g);
    } else if (HP2SPH_SWEEP_MB_MAX >= 2 && g.nmaps >= 2) {
        hipLaunchKernelGGL((k_sweep<T, 2, FWD>), dim3(sweep_workgroups(g, 2)), dim3(64 * SW_WAVES), 0, s, U, G, g);
    } else {
        hipLaunchKernelGGL((k_sweep<T, 1, FWD>), dim3(sweep_workgroups(g, 1)), dim3(64 * SW_WAVES), 0, s, U, G, g);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_sweep_fwd(Blocks4<T> U, Blocks4<const T> G, const GroupDims& g, hipStream_t s) {
    return launch_sweep<T, true>(U, G, g, s);
}

template <class T>
hipError_t launch_sweep_bwd(Blocks4<T> U, Blocks4<const T> G, const GroupDims& g, hipStream_t s) {
    return launch_sweep<T, false>(U, G, g, s);
}

// ---------------------------------------------------------------------------
// pack / unpack between U and the packed complex128 alm
// ---------------------------------------------------------------------------

// one thread per (block, map, l', k') complex entry; the fastest-varying index
// follows the column order of U (k' for map-major, map for mode-major) so
// that the U side is coalesced
__device__ __forceinline__ bool pack_index(const GroupDims& g, int blk, int64_t e, int& map, int& lp, int& kk) {
    const int nk = g.nk[blk], nl = g.nl[blk];
    if (e >= int64_t(nk) * nl * g.nmaps) return false;
    if (g.modemajor) {
        map = int(e % g.nmaps);
        const int64_t t = e / g.nmaps;
        kk = int(t % nk);
        lp = int(t / nk);
    } else {
        kk = int(e % nk);
        const int64_t t = e / nk;
        lp = int(t % nl);
        map = int(t / nl);
    }
    return true;
}

// Pack through an LDS tile: one workgroup per (order m, 64 consecutive l,
// 32 consecutive maps).  The two parity blocks of m (even and odd l) are
// read row by row (each row a contiguous run of maps in the mode-major
// layout) and every map's 64 a_l^m are written as one contiguous run of
// alm.  With Ub given, writes Ua + Ub (the refined a_lm), added in FP64.
// Tiles of 64 degrees and PM maps (PM = 16, 32 or 64: the tile shapes the
// autotuner chooses among; 32 by default).
constexpr int kPackL = 64, kPackMaps = 32;

// Pack tile `ti` (an (m, l0) pair of `tiles`) for the maps of map group `mg`.
template <class T, int kPackMaps>
__device__ __forceinline__ void pack_item(Quad<const T> Ua, Quad<const T> Ub, double* __restrict__ alm,
                                          const int64_t* __restrict__ alm_off, const int32_t* __restrict__ lmaxv,
                                          const int32_t* __restrict__ tiles, const GroupDims& g, int ti, int mg,
                                          C2<double> (*tile)[kPackMaps + 1]) {
    static_assert(kPackL * kPackMaps % 256 == 0, "a pack tile is a whole number of 256-thread sweeps");
    const int m = tiles[2 * ti], l0 = tiles[2 * ti + 1];
    const int v0 = mg * kPackMaps;
    const int kpar = m & 1, kk = m >> 1;
    const bool two = !Ub.null();
    // Branch-free, fully unrolled loads: an element outside the tile's maps or
    // degrees reads the tile's first element (map v0, degree l0, both in range)
    // and is dropped when the tile is filled, so all of a thread's loads are in
    // flight before the first of them is used.
    constexpr int kIt = kPackL * kPackMaps / 256;
    using P2 = typename Vec2<T>::type;   // one (re, im) pair
    P2 ra[kIt], rb[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int vi = i % kPackMaps, li = i / kPackMaps;
        const bool ok = v0 + vi < g.nmaps && l0 + li <= g.p;
        const int v = ok ? v0 + vi : v0, l = ok ? l0 + li : l0;
        // the block of order parity kpar whose l have the parity of l
        const int blk = 2 * kpar + ((l & 1) == (g.lmin[2 * kpar] & 1) ? 0 : 1);
        const int lp = (l - g.lmin[blk]) >> 1;
        const int64_t o = int64_t(lp) * g.N[kpar] + int64_t(v) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
        ra[it] = *reinterpret_cast<const P2*>(Ua.at(blk) + o);
        if (two) rb[it] = *reinterpret_cast<const P2*>(Ub.at(blk) + o);
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int vi = i % kPackMaps, li = i / kPackMaps;
        C2<double> z = {0.0, 0.0};
        if (v0 + vi < g.nmaps && l0 + li <= g.p) {
            z = {double(ra[it][0]), double(ra[it][1])};
            if (two) z = {z.x + double(rb[it][0]), z.y + double(rb[it][1])};
        }
        tile[li][vi] = z;
    }
    // the maps' band limits and alm offsets of the store phase, read while
    // the other lanes fill the tile
    int Ls[kIt];
    int64_t base[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int v = v0 + (threadIdx.x + 256 * it) / kPackL;
        const int vv = v < g.nmaps ? v : v0;
        Ls[it] = v < g.nmaps ? lmaxv[vv] : -1;
        base[it] = alm_off[vv];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int li = i % kPackL, vi = i / kPackL;
        const int l = l0 + li, L = Ls[it];
        if (l > L) continue;
        const int64_t o = 2 * (base[it] + int64_t(m) * (2 * L + 1 - m) / 2 + l);
        const C2<double> z = tile[li][vi];
        *reinterpret_cast<D2*>(alm + o) = D2{z.x, z.y};
    }
}

// Pack over the work list of every group of the launch: U of region reg_a
// (plus region reg_b when >= 0).  Items are (pack tile, map group) with the
// tile fastest; one workgroup per item.
template <class T, int PM>
__global__ __launch_bounds__(256) void k_pack(const GroupDesc* __restrict__ gd, GroupRange gr, char* ws, int reg_a,
                                              int reg_b, double* __restrict__ alm) {
    __shared__ C2<double> tile[kPackL][PM + 1];
    int gi, local;
    if (!locate_item(gr, blockIdx.x, gi, local)) return;
    const GroupDesc& G = gd[gi];
    const int nt = uniform(G.n_pack_tiles);
    pack_item<T, PM>(region_quad<const T>(ws, G, reg_a), region_quad<const T>(ws, G, reg_b), alm, uniform(G.alm_off),
                     uniform(G.lmax), uniform(G.pack_tiles), G.g, local % nt, local / nt, tile);
}

// Map-major layout (staged strategy): a map's orders of one parity are
// contiguous in each U row, so a tile is one map, 16 orders m0, m0 + 2, ..
// of one parity and 64 consecutive l: each row read is one contiguous run of
// 16 (re, im) pairs, each order's 64 a_l^m one contiguous run of alm.
constexpr int kPackOrders = 16;

template <class T>
__device__ __forceinline__ void pack_mm_item(Quad<const T> Ua, Quad<const T> Ub, double* __restrict__ alm,
                                             const int64_t* __restrict__ alm_off, const int32_t* __restrict__ lmaxv,
                                             const int32_t* __restrict__ tiles, const GroupDims& g, int ti, int v,
                                             C2<double> (*tile)[kPackOrders + 1]) {
    const int m0 = tiles[2 * ti], l0 = tiles[2 * ti + 1];
    const int kpar = m0 & 1, kk0 = m0 >> 1;
    const bool two = !Ub.null();
    const int p = g.p, lmin_even = g.lmin[2 * kpar];
    const int64_t N = g.N[kpar], colmap = int64_t(v) * g.cm[kpar], ck = g.ck[kpar];
    constexpr int kIt = kPackL * kPackOrders / 256;
    using P2 = typename Vec2<T>::type;
    P2 ra[kIt], rb[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int o = i % kPackOrders, li = i / kPackOrders;   // orders fastest: one contiguous run per row
        const int m = m0 + 2 * o, l = l0 + li;
        const bool ok = m <= p && l <= p;
        const int lq = ok ? l : l0, kk = ok ? kk0 + o : kk0;
        const int sel = (lq & 1) == (lmin_even & 1) ? 0 : 1;
        const int blk = 2 * kpar + sel;
        const int lp = (lq - g.lmin[blk]) >> 1;
        const int64_t off = int64_t(lp) * N + colmap + int64_t(kk) * ck;
        ra[it] = *reinterpret_cast<const P2*>(Ua.at(blk) + off);
        if (two) rb[it] = *reinterpret_cast<const P2*>(Ub.at(blk) + off);
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int o = i % kPackOrders, li = i / kPackOrders;
        C2<double> z = {double(ra[it][0]), double(ra[it][1])};
        if (two) z = {z.x + double(rb[it][0]), z.y + double(rb[it][1])};
        tile[li][o] = z;
    }
    const int L = lmaxv[v];
    const int64_t base = alm_off[v];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int li = i % kPackL, o = i / kPackL;   // degrees fastest: one contiguous run of alm per order
        const int m = m0 + 2 * o, l = l0 + li;
        if (m > L || l < m || l > L) continue;
        const int64_t at = 2 * (base + int64_t(m) * (2 * L + 1 - m) / 2 + l);
        const C2<double> z = tile[li][o];
        *reinterpret_cast<D2*>(alm + at) = D2{z.x, z.y};
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_pack_mm(const GroupDesc* __restrict__ gd, GroupRange gr, char* ws, int reg_a,
                                                 int reg_b, double* __restrict__ alm) {
    __shared__ C2<double> tile[kPackL][kPackOrders + 1];
    int gi, local;
    if (!locate_item(gr, blockIdx.x, gi, local)) return;
    const GroupDesc& G = gd[gi];
    const int nt = uniform(G.n_pack_tiles);
    pack_mm_item<T>(region_quad<const T>(ws, G, reg_a), region_quad<const T>(ws, G, reg_b), alm, uniform(G.alm_off),
                    uniform(G.lmax), uniform(G.pack_tiles), G.g, local % nt, local / nt, tile);
}

std::vector<int32_t> pack_tiles_mapmajor(int p) {
    std::vector<int32_t> t;
    for (int kpar = 0; kpar < 2; ++kpar)
        for (int m0 = kpar; m0 <= p; m0 += 2 * kPackOrders)
            for (int l0 = m0; l0 <= p; l0 += kPackL) {
                t.push_back(m0);
                t.push_back(l0);
            }
    return t;
}

std::vector<int32_t> pack_tiles(int p) {
    std::vector<int32_t> t;
    for (int m = 0; m <= p; ++m)
        for (int l0 = m; l0 <= p; l0 += kPackL) {
            t.push_back(m);
            t.push_back(l0);
        }
    return t;
}

// One launch per run of consecutive groups with the same column layout.
template <class T>
hipError_t launch_pack(const GroupLaunch& gl, int reg_a, int reg_b, double* alm, hipStream_t s) {
    for (int i = 0; i < gl.n;) {
        const bool mm = gl.host[gl.first + i].g.modemajor != 0;
        int j = i + 1;
        while (j < gl.n && (gl.host[gl.first + j].g.modemajor != 0) == mm) ++j;
        GroupLaunch run = gl;
        run.first = gl.first + i;
        run.n = j - i;
        GroupRange r;
        const int pm = gl.variant == 16 || gl.variant == 64 ? gl.variant : kPackMaps;
        hipError_t e = mm ? make_range(run,
                                       [pm](const GroupDesc& G) {
                                           return int64_t(G.n_pack_tiles) * ((G.g.nmaps + pm - 1) / pm);
                                       },
                                       r)
                          : make_range(run, [](const GroupDesc& G) { return int64_t(G.n_pack_tiles) * G.g.nmaps; }, r);
        if (e != hipSuccess) return e;
        if (r.start[r.n] > 0) {
            const dim3 grid(list_grid(run, r, false));
            if (mm && pm == 16)
                hipLaunchKernelGGL((k_pack<T, 16>), grid, dim3(256), 0, s, run.dev, r, run.ws, reg_a, reg_b, alm);
            else if (mm && pm == 64)
                hipLaunchKernelGGL((k_pack<T, 64>), grid, dim3(256), 0, s, run.dev, r, run.ws, reg_a, reg_b, alm);
            else if (mm)
                hipLaunchKernelGGL((k_pack<T, 32>), grid, dim3(256), 0, s, run.dev, r, run.ws, reg_a, reg_b, alm);
            else
                hipLaunchKernelGGL(k_pack_mm<T>, dim3(list_grid(run, r, false)), dim3(256), 0, s, run.dev, r, run.ws,
                                   reg_a, reg_b, alm);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        i = j;
    }
    return hipSuccess;
}

// U (FP32) -> U (FP64) in the same layout, zero where l < m or l > lmax of
// the column's map (what unpacking the packed a_lm would give).
// Widen item: row lp of block blk, pairs q0 + 2 t, q0 + 2 t + 1 (t the
// thread) of that row, each pair one FP32 (re, im) -> FP64 (re, im).
template <class BA, class BU>
__device__ __forceinline__ void widen_item(BA Ua, BU U, const int32_t* __restrict__ lmaxv, const GroupDims& g,
                                           int live_only, int blk, int lp, int q0) {
    const int kpar = blk >> 1;
    const int pairs = int(g.N[kpar] >> 1);
    const int l = g.lmin[blk] + 2 * lp;
    const int q = q0 + 2 * int(threadIdx.x);
    if (q >= pairs) return;
    const int64_t o = int64_t(lp) * g.N[kpar] + 2 * int64_t(q);
    const float* src = Ua.p[blk] + o;
    double* dst = U.p[blk] + o;
    const int nmaps = g.nmaps, per = g.Npm[kpar] >> 1, nk = g.nk[blk];
    // the two pairs' (map, k'): consecutive maps of one mode (mode-major) or
    // consecutive modes of one map (map-major)
    int map0, kk0;
    if (g.modemajor) {
        kk0 = q / nmaps;
        map0 = q - kk0 * nmaps;
    } else {
        map0 = q / per;
        kk0 = q - map0 * per;
    }
    const bool two = q + 1 < pairs;
    // two 8-byte loads: a row of an odd-width block starts 8 bytes off a
    // 16-byte boundary
    const float2 v0 = *reinterpret_cast<const float2*>(src);
    const float2 v1 = two ? *reinterpret_cast<const float2*>(src + 2) : make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (i == 1 && !two) break;
        int map = map0, kk = kk0;
        if (i == 1) {
            if (g.modemajor) {
                if (++map == nmaps) { map = 0; ++kk; }
            } else {
                if (++kk == per) { kk = 0; ++map; }
            }
        }
        const int m = 2 * kk + kpar;
        if (live_only && l < m) continue;   // rows below the order are never read
        D2 w = {0.0, 0.0};
        if (kk < nk && l >= m && l <= lmaxv[map])
            w = i == 0 ? D2{double(v0.x), double(v0.y)} : D2{double(v1.x), double(v1.y)};
        *reinterpret_cast<D2*>(dst + 2 * i) = w;
    }
}

// Widen items of a group: 4 blocks x (largest block's rows) x (512-pair
// chunks of the longest row), the ranges of a smaller block padded.
__host__ __device__ inline int widen_chunks(const GroupDims& g) {
    const int64_t most = g.N[0] > g.N[1] ? g.N[0] : g.N[1];
    return int((most / 2 + 511) / 512);
}
__host__ __device__ inline int widen_rows(const GroupDims& g) {
    int r = 0;
    for (int b = 0; b < 4; ++b) r = r > g.nl[b] ? r : g.nl[b];
    return r;
}

// Widen over the work list of every group (region Ua -> region U).
__global__ __launch_bounds__(256) void k_widen(const GroupDesc* __restrict__ gd, GroupRange gr, char* ws) {
    int gi, local;
    if (!locate_item(gr, blockIdx.x, gi, local)) return;
    const GroupDesc& G = gd[gi];
    const int ch = widen_chunks(G.g), rows = widen_rows(G.g);
    const int blk = local / (rows * ch);
    const int rem = local - blk * rows * ch;
    const int lp = rem / ch, c = rem - lp * ch;
    if (lp >= G.g.nl[blk]) return;
    widen_item(region_blocks<const float>(ws, G, kRegUa), region_blocks<double>(ws, G, kRegU), G.lmax, G.g,
               G.tables, blk, lp, c * 512);
}

hipError_t launch_widen(const GroupLaunch& gl, hipStream_t s) {
    GroupRange r;
    if (hipError_t e = make_range(
            gl, [](const GroupDesc& G) { return int64_t(4) * widen_rows(G.g) * widen_chunks(G.g); }, r);
        e != hipSuccess)
        return e;
    if (r.start[r.n] == 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3(list_grid(gl, r, false)), dim3(256), 0, s, gl.dev, r, gl.ws);
    return hipGetLastError();
}

// Jacobi update in the U layout (per-order tables, mode-major):
// Uacc = (first ? 0 : Uacc) + U for the live entries m <= l <= lmax of each
// column's map, zero for l > lmax (the synthesis reads a truncated at lmax);
// rows l < m are never read and stay untouched.
__global__ void k_accumulate(Blocks4<const double> U, Blocks4<double> Uacc, const int32_t* __restrict__ lmaxv,
                             GroupDims g, int first) {
    const int blk = blockIdx.y, kpar = blk >> 1;
    const int64_t pairs = g.N[kpar] >> 1;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(g.nl[blk]) * pairs) return;
    const int lp = int(e / pairs);
    const int64_t q = e % pairs;
    const int kk = int(q / g.nmaps), map = int(q % g.nmaps);
    const int l = g.lmin[blk] + 2 * lp, m = 2 * kk + kpar;
    if (kk >= g.nk[blk] || l < m) return;
    const int64_t o = int64_t(lp) * g.N[kpar] + 2 * q;
    D2 v = {0.0, 0.0};
    if (l <= lmaxv[map]) {
        const D2 u = *reinterpret_cast<const D2*>(U.p[blk] + o);
        v = u;
        if (!first) {
            const D2 w = *reinterpret_cast<const D2*>(Uacc.p[blk] + o);
            v = {w.x + u.x, w.y + u.y};
        }
    }
    *reinterpret_cast<D2*>(Uacc.p[blk] + o) = v;
}

hipError_t launch_accumulate(Blocks4<const double> U, Blocks4<double> Uacc, const int32_t* lmax, const GroupDims& g,
                             bool first, hipStream_t s) {
    if (!g.modemajor) return hipErrorInvalidValue;
    int64_t most = 0;
    for (int b = 0; b < 4; ++b) most = std::max<int64_t>(most, int64_t(g.nl[b]) * (g.N[b >> 1] >> 1));
    hipLaunchKernelGGL(k_accumulate, dim3(unsigned((most + 255) / 256), 4), dim3(256), 0, s, U, Uacc, lmax, g,
                       first ? 1 : 0);
    return hipGetLastError();
}

static dim3 pack_grid(const GroupDims& g) {
    int64_t most = 0;
    for (int b = 0; b < 4; ++b) most = std::max<int64_t>(most, int64_t(g.nk[b]) * g.nl[b] * g.nmaps);
    return dim3(unsigned((most + 255) / 256), 4);
}

__global__ void k_unpack(const double* __restrict__ alm, const int64_t* __restrict__ alm_off,
                         const int32_t* __restrict__ lmaxv, Blocks4<double> U, GroupDims g) {
    const int blk = blockIdx.y;
    const int kpar = blk >> 1;
    int map, lp, kk;
    if (!pack_index(g, blk, int64_t(blockIdx.x) * blockDim.x + threadIdx.x, map, lp, kk)) return;
    const int l = g.lmin[blk] + 2 * lp, m = 2 * kk + kpar;
    const int L = lmaxv[map];
    double re = 0.0, im = 0.0;
    if (l >= m && l <= L) {
        const int64_t o = 2 * (alm_off[map] + int64_t(m) * (2 * L + 1 - m) / 2 + l);
        re = alm[o];
        im = alm[o + 1];
    }
    double* dst = U.p[blk] + int64_t(lp) * g.N[kpar] + int64_t(map) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
    dst[0] = re;
    dst[1] = im;
}

hipError_t launch_unpack(const double* alm, const int64_t* alm_off, const int32_t* lmax, Blocks4<double> U,
                         const GroupDims& g, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack, pack_grid(g), dim3(256), 0, s, alm, alm_off, lmax, U, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis: inverse ring transform (+ residual)
// ---------------------------------------------------------------------------

// Mode sums of one ring from Dsym row h: with D_k = D+_k + sgn D-_k and
// G_k = D_k e^{i k phi0} (k = 0..p), leaves in buf[lpad(t)], t = 0..n/2,
//   H_t = sum_{k = t mod n} G_k + conj(sum_{k > 0, k = -t mod n} G_k),
// the DFT coefficients (up to the factor n) of the real ring values the
// coefficients D_k take at the ring's n points (modes |k| >= n alias).
// For a shifted ring (phi0 = pi / n) the phase factors out of the alias
// chains: e^{i pi (t + a n) / n} = (-1)^a e^{i pi t / n}, so
//   H_t = e^{i pi t / n} (A_t - conj B_t),  A_t = sum_a (-1)^a D_{t + a n},
//   B_t = sum_a (-1)^a D_{n - t + a n};  unshifted: H_t = A_t + conj B_t
// without the signs.  D_k is staged in buf[0..p] (coalesced loads), partial
// chain sums in buf[p+1 ..]; buf needs p + 1 + NT slots.  Ends with a barrier.
template <int NT>
__device__ __forceinline__ void ring_mode_sums(const Blocks4<const double>& D, int h, int sgn, int n, bool shifted,
                                               int p, const GroupDims& g, int map, const double* roots,
                                               C2<double>* buf) {
    const int L = n >> 1, T1 = L + 1;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kRingKPT; ++i) {
        const int k = tid + i * NT;
        if (k <= p) {
            const int kpar = k & 1, kk = k >> 1;
            const int64_t o = int64_t(h) * g.N[kpar] + int64_t(map) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
            const D2 vp = *reinterpret_cast<const D2*>(D.p[2 * kpar] + o);
            const D2 vm = *reinterpret_cast<const D2*>(D.p[2 * kpar + 1] + o);
            buf[lpad(k)] = {vp.x + sgn * vm.x, vp.y + sgn * vm.y};
        }
    }
    __syncthreads();
    // sum over a = s, s + c, s + 2c, ... of (+-1)^a D_{k0 + a n}
    auto chain = [&](int k0, int s, int c) -> C2<double> {
        C2<double> acc = {0.0, 0.0};
        for (int a = s, k = k0 + s * n; k <= p; a += c, k += c * n) {
            const C2<double> v = buf[lpad(k)];
            acc = (shifted && (a & 1)) ? csub(acc, v) : cadd(acc, v);
        }
        return acc;
    };
    auto combine = [&](int t, int s, int c) -> C2<double> {
        const C2<double> A = chain(t, s, c), B = chain(n - t, s, c);
        return shifted ? csub(A, cconj(B)) : cadd(A, cconj(B));
    };
    auto phase = [&](C2<double> v, int t) -> C2<double> {
        return shifted ? cmul(v, cconj(ldc(roots, t))) : v;   // e^{+i pi t / n}
    };
    const int c = NT / T1;
    if (c > 1) {
        // c threads per t, partial sums added in a fixed order
        C2<double> part = {0.0, 0.0};
        if (tid < c * T1) part = combine(tid % T1, tid / T1, c);
        buf[lpad(p + 1 + tid)] = part;
        __syncthreads();
        if (tid < T1) {
            C2<double> hs = {0.0, 0.0};
            for (int s = 0; s < c; ++s) hs = cadd(hs, buf[lpad(p + 1 + s * T1 + tid)]);
            buf[lpad(tid)] = phase(hs, tid);   // D_k is no longer read: the chains ended at the barrier
        }
    } else {
        C2<double> H[kRingKPT];
#pragma unroll
        for (int i = 0; i < kRingKPT; ++i) {
            const int t = tid + i * NT;
            H[i] = (t < T1) ? phase(combine(t, 0, 1), t) : C2<double>{0.0, 0.0};
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kRingKPT; ++i) {
            const int t = tid + i * NT;
            if (t < T1) buf[lpad(t)] = H[i];
        }
    }
    __syncthreads();
}

// One ring of the synthesis: values x_q, q < n, of the real trigonometric
// polynomial with coefficients D_k = D+_k + sgn D-_k, k = 0..p (and the
// conjugates at -k), evaluated at lambda_q = phi0 + 2 pi q / n.  Modes |k| >= n
// alias onto k mod n.  Written to out (minus minus_from[q] - x_q if given).
template <int NT>
__device__ __forceinline__ void ring_synth(const Blocks4<const double>& D, int h, int sgn, int n, bool shifted, int p,
                                           const GroupDims& g, int map, FftTab<double> ft, C2<double>* buf,
                                           double* out, const double* minus_from) {
    const int L = n >> 1, j = n >> 2;
    const int Mb = ft.chirpm[j];
    const double* roots = ft.roots + 2 * ft.rootoff[j];
    ring_mode_sums<NT>(D, h, sgn, n, shifted, p, g, map, roots, buf);
    // Z'_t = (H_t + conj H_{L-t}) + i (H_t - conj H_{L-t}) e^{2 pi i t / n}, t < L;
    // x_{2q} + i x_{2q+1} = sum_t Z'_t e^{2 pi i t q / L}, computed as conj(DFT(conj Z')).
    auto src = [&](int t) -> C2<double> {
        const C2<double> ht = buf[lpad(t)], hl = buf[lpad(L - t)];
        const C2<double> e = cadd(ht, cconj(hl));
        const C2<double> o = cmul(csub(ht, cconj(hl)), cconj(ldc(roots, 2 * t)));
        const C2<double> z = {e.x - o.y, e.y + o.x};
        return cconj(z);
    };
    const double* chirp = ft.chirp + 2 * ft.chirpoff[j];
    const double* chirpfft = ft.chirpfft + 2 * ft.chirpfftoff[j];
    const DftOut<double> R =
        ring_dft<double, NT, kRingMaxV>(buf, L, Mb, chirp, chirpfft, ft.twiddle, ft.fft_max, src);
    for (int q = threadIdx.x; q < L; q += NT) {
        const C2<double> z = cconj(R.Z(q));
        D2 v = {z.x, z.y};
        if (minus_from) {
            const D2 f = *reinterpret_cast<const D2*>(minus_from + 2 * q);
            v = {f.x - v.x, f.y - v.y};
        }
        *reinterpret_cast<D2*>(out + 2 * q) = v;
    }
    __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_ring_inverse(Blocks4<const double> D, RingTab rt, FftTab<double> ft,
                                                     double* out, const double* minus_from,
                                                     const int64_t* __restrict__ map_off, GroupDims g) {
    extern __shared__ unsigned char smem_raw[];
    C2<double>* buf = reinterpret_cast<C2<double>*>(smem_raw);
    int map, h;
    ring_block(g.nmaps, 2 * g.nside, map, h);
    const int ns = g.nside;
    const int64_t mo = map_off[map];
    {
        const int r0 = h - 1;
        const int64_t st = mo + rt.start[r0];
        ring_synth<NT>(D, h, +1, rt.n[r0], rt.shifted[r0] != 0, g.p, g, map, ft, buf, out + st,
                       minus_from ? minus_from + st : nullptr);
    }
    if (h < 2 * ns) {
        const int r0 = 4 * ns - h - 1;
        const int64_t st = mo + rt.start[r0];
        ring_synth<NT>(D, h, -1, rt.n[r0], rt.shifted[r0] != 0, g.p, g, map, ft, buf, out + st,
                       minus_from ? minus_from + st : nullptr);
    }
}

hipError_t launch_ring_inverse(Blocks4<const double> D, RingTab rt, FftTab<double> ft, double* out,
                               const double* minus_from, const int64_t* map_off, const GroupDims& g,
                               hipStream_t s) {
    dim3 grid(g.nmaps, 2 * g.nside);
    const int nt = ring_threads(ft.fft_max);
    const size_t shm = lds_slots_bytes(std::max(ft.fft_max, g.p + 1 + nt), sizeof(C2<double>));
    if (nt == 256)
        hipLaunchKernelGGL(k_ring_inverse<256>, grid, dim3(256), shm, s, D, rt, ft, out, minus_from, map_off, g);
    else
        hipLaunchKernelGGL(k_ring_inverse<512>, grid, dim3(512), shm, s, D, rt, ft, out, minus_from, map_off, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Refinement residual in ring-Fourier space
// ---------------------------------------------------------------------------
//
// For the maps' FP64 ring coefficients Df (Dsym rows 1..2 nside, as the
// forward ring transform writes them) and the synthesis GEMM output Gs (the
// same rows of S a0 before the inverse ring transform), writes
//   Dr = Df - Ring(Synth(Gs))
// in FP32.  Ring(Synth(.)) of one ring with n points, L = n/2, is exact
// arithmetic on the coefficients (no FFT): the inverse transform folds the
// modes k = 0..p onto the ring's DFT bins and the forward transform reads the
// bins back, so
//   X_k = A_k + conj B_k (unshifted ring) or A_k - conj B_k (shifted),  k < L,
//   A_k = sum_a s_a D_{k + a n},  B_k = sum_a s_a D_{n - k + a n},
//   s_a = 1 (unshifted) or (-1)^a (shifted: the half-pixel phase e^{i pi k/n}
//   turns into these signs and cancels against the forward shift),
// X_L from the forward transform's Nyquist rule with alpha the (real)
// Nyquist bin of the synthesized ring (Re X'_L, or -Im X'_L for a shifted
// ring, X'_L = the k = L instance of the formula above), and X_k = 0 above L.
// The N and S rings of a pair share n and the shift, and D_k = D+ +- D-, so
// one pass over the aliases gives both.
//
// A workgroup takes one ring pair of 16 consecutive maps; lane bits 0..3 pick
// the map, so that in the mode-major layout every access to one (row, mode)
// is one contiguous run of 16 maps.

constexpr int kFoldMaps = 16;
// Maps per fold workgroup: 16 consecutive maps share a (row, mode) run in the
// mode-major layout; in the map-major layout (staged strategy) a map's modes
// are contiguous, so there a workgroup takes one map and its lanes walk
// consecutive modes.
__host__ __device__ inline int fold_maps(const GroupDims& g) { return g.modemajor ? kFoldMaps : 1; }

// Work item `id` of one group: ring pair h of map group mg (ring_block_id).
template <int NT, class BD, class BR>
__device__ __forceinline__ void residual_fold_item(BD Df, BD Gs, BR Dr, const RingTab& rt, const GroupDims& g, int id,
                                                   C2<double>* partN, C2<double>* partS) {
    const int FM = fold_maps(g);          // maps per workgroup (16 or 1)
    const int SL = NT / FM;               // k slots per map
    const int mgroups = (g.nmaps + FM - 1) / FM;
    int mg, h;
    ring_block_id(id, mgroups, 2 * g.nside, mg, h);
    const int m8 = threadIdx.x % FM, slot = threadIdx.x / FM;
    const int map = mg * FM + m8;
    const bool valid = map < g.nmaps;
    const int ns = g.nside, p = g.p;
    const bool equator = (h == 2 * ns);
    const int n = rt.n[h - 1], L = n >> 1, T1 = L + 1;
    const bool shifted = rt.shifted[h - 1] != 0;
    auto offs = [&](int k) -> int64_t {
        const int kpar = k & 1, kk = k >> 1;
        return int64_t(h) * g.N[kpar] + int64_t(map) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
    };
    // alias chains from a = s in steps of c of both rings
    auto chains = [&](int t, int s, int c, C2<double>& SN, C2<double>& SS) {
        C2<double> Ap = {0.0, 0.0}, Am = {0.0, 0.0}, Bp = {0.0, 0.0}, Bm = {0.0, 0.0};
        if (valid) {
            for (int a = s, k = t + s * n; k <= p; a += c, k += c * n) {
                const int64_t o = offs(k);
                const D2 vp = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1)] + o);
                const D2 vm = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1) + 1] + o);
                const double sg = (shifted && (a & 1)) ? -1.0 : 1.0;
                Ap = {Ap.x + sg * vp.x, Ap.y + sg * vp.y};
                Am = {Am.x + sg * vm.x, Am.y + sg * vm.y};
            }
            for (int a = s, k = n - t + s * n; k <= p; a += c, k += c * n) {
                const int64_t o = offs(k);
                const D2 vp = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1)] + o);
                const D2 vm = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1) + 1] + o);
                const double sg = (shifted && (a & 1)) ? -1.0 : 1.0;
                Bp = {Bp.x + sg * vp.x, Bp.y + sg * vp.y};
                Bm = {Bm.x + sg * vm.x, Bm.y + sg * vm.y};
            }
        }
        const C2<double> AN = cadd(Ap, Am), BN = cadd(Bp, Bm), AS = csub(Ap, Am), BS = csub(Bp, Bm);
        SN = shifted ? csub(AN, cconj(BN)) : cadd(AN, cconj(BN));
        SS = shifted ? csub(AS, cconj(BS)) : cadd(AS, cconj(BS));
    };
    // X_k of one ring from its chain value at k (k <= L)
    auto coeff = [&](int k, C2<double> S) -> C2<double> {
        if (k < L) return S;
        const double alpha = shifted ? -S.y : S.x;
        if (L < p) return {0.0, -0.5 * alpha};
        return {shifted ? 0.0 : 0.5 * alpha, 0.0};
    };
    auto emit = [&](int k, C2<double> XN, C2<double> XS) {
        if (!valid) return;
        C2<double> sp, sm;
        if (equator) {
            sp = XN;
            sm = {0.0, 0.0};
        } else {
            sp = cscale(cadd(XN, XS), 0.5);
            sm = cscale(csub(XN, XS), 0.5);
        }
        const int64_t o = offs(k);
        const int kpar = k & 1;
        const D2 fp = *reinterpret_cast<const D2*>(Df.p[2 * kpar] + o);
        const D2 fm = *reinterpret_cast<const D2*>(Df.p[2 * kpar + 1] + o);
        float* rp = Dr.p[2 * kpar];
        float* rm = Dr.p[2 * kpar + 1];
        rp[o] = float(fp.x - sp.x);
        rp[o + 1] = float(fp.y - sp.y);
        rm[o] = float(fm.x - sm.x);
        rm[o + 1] = float(fm.y - sm.y);
    };
    const C2<double> zero = {0.0, 0.0};
    const int c = SL / T1;
    if (c > 1) {
        // short rings: c slots per bin, partial sums added in a fixed order
        C2<double> SN = zero, SS = zero;
        if (slot < c * T1) chains(slot % T1, slot / T1, c, SN, SS);
        partN[threadIdx.x] = SN;
        partS[threadIdx.x] = SS;
        __syncthreads();
        if (slot < T1) {
            C2<double> hn = zero, hs = zero;
            for (int q = 0; q < c; ++q) {
                hn = cadd(hn, partN[(q * T1 + slot) * FM + m8]);
                hs = cadd(hs, partS[(q * T1 + slot) * FM + m8]);
            }
            emit(slot, coeff(slot, hn), coeff(slot, hs));
        }
        for (int k = T1 + slot; k <= p; k += SL) emit(k, zero, zero);
    } else {
        // Bins with a single alias and no mirror term (n > p, k < min(L, n - p)):
        // X_k = D_k on both rings, so Dr = Df - Gs element by element (on the
        // equator Gs- and Df- are zero).  This covers most of every row.
        const int k_simple = (n > p) ? min(L, n - p) : 0;
        int k = slot;
        if (valid) {
#pragma unroll 4
            for (; k < k_simple; k += SL) {
                const int64_t o = offs(k);
                const int kp = k & 1;
                const D2 gp = *reinterpret_cast<const D2*>(Gs.p[2 * kp] + o);
                const D2 gm = *reinterpret_cast<const D2*>(Gs.p[2 * kp + 1] + o);
                const D2 fp = *reinterpret_cast<const D2*>(Df.p[2 * kp] + o);
                const D2 fm = *reinterpret_cast<const D2*>(Df.p[2 * kp + 1] + o);
                *reinterpret_cast<F2*>(Dr.p[2 * kp] + o) = F2{float(fp.x - gp.x), float(fp.y - gp.y)};
                *reinterpret_cast<F2*>(Dr.p[2 * kp + 1] + o) = F2{float(fm.x - gm.x), float(fm.y - gm.y)};
            }
        } else {
            while (k < k_simple) k += SL;
        }
        for (; k <= p; k += SL) {
            if (k <= L) {
                C2<double> SN, SS;
                chains(k, 0, 1, SN, SS);
                emit(k, coeff(k, SN), coeff(k, SS));
            } else {
                emit(k, zero, zero);
            }
        }
    }
}

// The fold over the work list of every group (regions Df and D -> Dr), one
// workgroup per item or (PERSIST) a grid that walks the list with a barrier
// between items (a candidate the autotuner measures).
template <int NT>
__device__ __forceinline__ void residual_fold_list_item(const GroupDesc* __restrict__ gd, const GroupRange& gr,
                                                        char* ws, int id, C2<double>* partN, C2<double>* partS) {
    int gi, local;
    if (!locate_item(gr, id, gi, local)) return;
    const GroupDesc& G = gd[gi];
    residual_fold_item<NT>(region_blocks<const double>(ws, G, kRegDf), region_blocks<const double>(ws, G, kRegD),
                           region_blocks<float>(ws, G, kRegDr), G.rt, G.g, local, partN, partS);
}

template <int NT, bool PERSIST>
__global__ __launch_bounds__(NT) void k_residual_fold(const GroupDesc* __restrict__ gd, GroupRange gr, char* ws) {
    __shared__ C2<double> partN[NT], partS[NT];
    if constexpr (PERSIST) {
        const int total = gr.start[gr.n];
        for (int id = blockIdx.x; id < total; id += gridDim.x) {
            residual_fold_list_item<NT>(gd, gr, ws, id, partN, partS);
            __syncthreads();
        }
    } else {
        residual_fold_list_item<NT>(gd, gr, ws, blockIdx.x, partN, partS);
    }
}

hipError_t launch_residual_fold(const GroupLaunch& gl, hipStream_t s) {
    GroupRange r;
    if (hipError_t e = make_range(
            gl,
            [](const GroupDesc& G) {
                return int64_t((G.g.nmaps + fold_maps(G.g) - 1) / fold_maps(G.g)) * 2 * G.g.nside;
            },
            r);
        e != hipSuccess)
        return e;
    if (r.start[r.n] == 0) return hipSuccess;
    const unsigned grid = list_grid(gl, r, true);
    if (int64_t(grid) < int64_t(r.start[r.n]))
        hipLaunchKernelGGL((k_residual_fold<256, true>), dim3(grid), dim3(256), 0, s, gl.dev, r, gl.ws);
    else
        hipLaunchKernelGGL((k_residual_fold<256, false>), dim3(grid), dim3(256), 0, s, gl.dev, r, gl.ws);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Equal-weight iteration: the residual's longitude sums in ring-Fourier space
// ---------------------------------------------------------------------------
//
// For the weighted longitude sums Wf of the maps (k_ring_adjoint) and the
// synthesis GEMM output Gs (coefficients D_k, k = 0..p, of S a per ring pair,
// D_{-k} = conj D_k), writes Wr = Wf - W(S a) for Dsym rows 1 .. 2 nside: the
// longitude sums of the synthesized ring x_q = sum_{|k| <= p} D_k e^{i k
// lambda_q} follow from the coefficients without a transform,
//   F(m) = sum_q x_q e^{-i m lambda_q} = n sum_{k = m mod n} D_k e^{i (k-m) phi0}
//        = n s^q (A_t + s conj B_t),   t = m mod n, q = m div n,
//   A_t = sum_b s^b D_{t + b n},  B_t = sum_b s^b D_{n - t + b n}  (indices <= p),
// s = -1 on a shifted ring (phi0 = pi / n), 1 otherwise.  Each bin t is
// summed once and written to every m = t + q n <= p.  Rings with n > p need
// only t = m, with at most one mirror term.  N and S rings share n and the
// shift, and D_k = D+ +- D-, so one pass gives both; then
// W+- = scale (F_N +- F_S) (equator: scale F_N, 0) as in k_ring_adjoint.
// Layout and workgroup shape as k_residual_fold: one ring pair of 16
// consecutive maps, lane bits 0..3 pick the map.
template <int NT>
__global__ __launch_bounds__(NT) void k_adjoint_residual(Blocks4<const double> Wf, Blocks4<const double> Gs,
                                                         Blocks4<double> Wr, RingTab rt, GroupDims g,
                                                         double scale) {
    constexpr int SL = NT / kFoldMaps;   // bin slots per map
    const int mgroups = (g.nmaps + kFoldMaps - 1) / kFoldMaps;
    int mg, h;
    ring_block(mgroups, 2 * g.nside, mg, h);
    const int m8 = threadIdx.x % kFoldMaps, slot = threadIdx.x / kFoldMaps;
    const int map = mg * kFoldMaps + m8;
    if (map >= g.nmaps) return;   // no barriers below
    const int ns = g.nside, p = g.p;
    const bool equator = (h == 2 * ns);
    const int n = rt.n[h - 1];
    const bool shifted = rt.shifted[h - 1] != 0;
    const double s = shifted ? -1.0 : 1.0;
    const double dn = double(n);
    auto offs = [&](int k) -> int64_t {
        const int kpar = k & 1, kk = k >> 1;
        return int64_t(h) * g.N[kpar] + int64_t(map) * g.cm[kpar] + int64_t(kk) * g.ck[kpar];
    };
    // D_k of the north and south rings
    auto coef = [&](int k, C2<double>& dN, C2<double>& dS) {
        const int64_t o = offs(k);
        const D2 vp = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1)] + o);
        const D2 vm = *reinterpret_cast<const D2*>(Gs.p[2 * (k & 1) + 1] + o);
        dN = {vp.x + vm.x, vp.y + vm.y};
        dS = {vp.x - vm.x, vp.y - vm.y};
    };
    // Wr at mode m from the ring sums F_N, F_S
    auto emit = [&](int m, C2<double> FN, C2<double> FS) {
        C2<double> wp, wm;
        if (equator) {
            wp = cscale(FN, scale);
            wm = {0.0, 0.0};
        } else {
            wp = cscale(cadd(FN, FS), scale);
            wm = cscale(csub(FN, FS), scale);
        }
        const int64_t o = offs(m);
        const int kpar = m & 1;
        const D2 fp = *reinterpret_cast<const D2*>(Wf.p[2 * kpar] + o);
        const D2 fm = *reinterpret_cast<const D2*>(Wf.p[2 * kpar + 1] + o);
        *reinterpret_cast<D2*>(Wr.p[2 * kpar] + o) = D2{fp.x - wp.x, fp.y - wp.y};
        *reinterpret_cast<D2*>(Wr.p[2 * kpar + 1] + o) = D2{fm.x - wm.x, fm.y - wm.y};
    };
    if (n > p) {
        // t = m; A_m = D_m, B_m = D_{n - m} when n - m <= p
        for (int m = slot; m <= p; m += SL) {
            C2<double> XN, XS;
            coef(m, XN, XS);
            if (n - m <= p) {
                C2<double> bN, bS;
                coef(n - m, bN, bS);
                XN = cadd(XN, cscale(cconj(bN), s));
                XS = cadd(XS, cscale(cconj(bS), s));
            }
            emit(m, cscale(XN, dn), cscale(XS, dn));
        }
    } else {
        for (int t = slot; t < n; t += SL) {
            C2<double> AN = {0.0, 0.0}, AS = {0.0, 0.0}, BN = {0.0, 0.0}, BS = {0.0, 0.0};
            double sg = 1.0;
            for (int k = t; k <= p; k += n, sg *= s) {
                C2<double> dN, dS;
                coef(k, dN, dS);
                AN = cadd(AN, cscale(dN, sg));
                AS = cadd(AS, cscale(dS, sg));
            }
            sg = 1.0;
            for (int k = n - t; k <= p; k += n, sg *= s) {
                C2<double> dN, dS;
                coef(k, dN, dS);
                BN = cadd(BN, cscale(dN, sg));
                BS = cadd(BS, cscale(dS, sg));
            }
            const C2<double> XN = cadd(AN, cscale(cconj(BN), s));
            const C2<double> XS = cadd(AS, cscale(cconj(BS), s));
            double sq = dn;
            for (int m = t; m <= p; m += n, sq *= s) emit(m, cscale(XN, sq), cscale(XS, sq));
        }
    }
}

hipError_t launch_adjoint_residual(Blocks4<const double> Wf, Blocks4<const double> Gs, Blocks4<double> Wr, RingTab rt,
                                   const GroupDims& g, double scale, hipStream_t s) {
    const int mgroups = (g.nmaps + kFoldMaps - 1) / kFoldMaps;
    dim3 grid(mgroups, 2 * g.nside);
    hipLaunchKernelGGL(k_adjoint_residual<256>, grid, dim3(256), 0, s, Wf, Gs, Wr, rt, g, scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// S5: C_l
// ---------------------------------------------------------------------------

// One workgroup per (32 consecutive l, map); 8 groups of 32 lanes split the
// orders m = 0..l into 8 contiguous ranges (lanes of a group read 32
// consecutive a_l^m of one order), and the 8 partial sums are added in a
// fixed order, so C_l is bitwise reproducible.
constexpr int kClL = 32, kClParts = 8;

__global__ __launch_bounds__(kClL * kClParts) void k_cl(const double* __restrict__ alm,
                                                        const int64_t* __restrict__ alm_off,
                                                        const int32_t* __restrict__ lmaxv, double* __restrict__ cl,
                                                        const int64_t* __restrict__ cl_off) {
    __shared__ double part[kClParts][kClL];
    const int map = blockIdx.y;
    const int L = lmaxv[map];
    const int li = threadIdx.x % kClL, c = threadIdx.x / kClL;
    const int l = blockIdx.x * kClL + li;
    const int span = (L + kClParts) / kClParts;            // ceil((L + 1) / parts)
    double s = 0.0;
    if (l <= L) {
        const double* a = alm + 2 * alm_off[map];
        const int m_end = min(l, (c + 1) * span - 1);
        for (int m = c * span; m <= m_end; ++m) {
            const int64_t o = 2 * (int64_t(m) * (2 * L + 1 - m) / 2 + l);
            const double re = a[o], im = a[o + 1];
            const double v = re * re + im * im;
            s += (m == 0) ? v : 2.0 * v;
        }
    }
    part[c][li] = s;
    __syncthreads();
    if (c == 0 && l <= L) {
        double t = part[0][li];
        for (int q = 1; q < kClParts; ++q) t += part[q][li];
        cl[cl_off[map] + l] = t / (2.0 * l + 1.0);
    }
}

hipError_t launch_cl(const double* alm, const int64_t* alm_off, const int32_t* lmax, double* cl,
                     const int64_t* cl_off, int nmaps, int lmax_max, hipStream_t s) {
    dim3 grid(unsigned((lmax_max + kClL) / kClL), nmaps);
    hipLaunchKernelGGL(k_cl, grid, dim3(kClL * kClParts), 0, s, alm, alm_off, lmax, cl, cl_off);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static workspace of the allocation-free analysis (hp2sph_analyze_noalloc)
// ---------------------------------------------------------------------------

// A file-scope device array: every device the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is looked up per device
// with hipGetSymbolAddress (scratch_init) and only that address is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
    return hipSuccess;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

hipError_t configure_kernels() {
    const int bytes = 160 * 1024;
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_ring_forward<256, 16>),
        reinterpret_cast<const void*>(&k_ring_forward<512, 16>),
        reinterpret_cast<const void*>(&k_ring_forward<512, 8>),
        reinterpret_cast<const void*>(&k_ring_inverse<256>),
        reinterpret_cast<const void*>(&k_ring_inverse<512>),
        reinterpret_cast<const void*>(&k_ring_adjoint<256>),
        reinterpret_cast<const void*>(&k_ring_adjoint<512>),

    };
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// explicit instantiations
template hipError_t launch_pole<double>(const GroupLaunch&, int, hipStream_t);
template hipError_t launch_pole<float>(const GroupLaunch&, int, hipStream_t);
template hipError_t launch_gemm<double, double>(const GemmProblem<double>*, const int32_t*, int, const double*,
                                               double*, hipStream_t);
template hipError_t launch_gemm<float, float>(const GemmProblem<float>*, const int32_t*, int, const float*, float*,
                                             hipStream_t);
template hipError_t launch_gemm<float, double>(const GemmProblem<float>*, const int32_t*, int, const double*, float*,
                                              hipStream_t);
template std::vector<int32_t> xcd_tile_map<double>(const GemmProblem<double>*, int);
template std::vector<int32_t> xcd_tile_map<float>(const GemmProblem<float>*, int);
template int finalize_gemm_problems<double>(GemmProblem<double>*, int);
template int finalize_gemm_problems<float>(GemmProblem<float>*, int);
template hipError_t launch_replicate<double>(const double*, int64_t, int64_t, int, int, int, double*, int, int,
                                             hipStream_t);
template hipError_t launch_scatter_tables<double>(const double*, int, int, int, int, int, const int64_t*,
                                                  const int32_t*, int, bool, double*, hipStream_t);
template hipError_t launch_sweep_fwd<double>(Blocks4<double>, Blocks4<const double>, const GroupDims&, hipStream_t);
template hipError_t launch_sweep_fwd<float>(Blocks4<float>, Blocks4<const float>, const GroupDims&, hipStream_t);
template hipError_t launch_sweep_bwd<double>(Blocks4<double>, Blocks4<const double>, const GroupDims&, hipStream_t);
template hipError_t launch_pack<double>(const GroupLaunch&, int, int, double*, hipStream_t);
template hipError_t launch_pack<float>(const GroupLaunch&, int, int, double*, hipStream_t);

}  // namespace hp2sph
