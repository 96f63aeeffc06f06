// Host-side FP64 set-up tables (see tables.h).  Built once per plan; nothing
// here runs per call.
#include "tables.h"

#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <thread>

namespace hp2sph {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

template <class F>
void parallel_for(int64_t n, F&& fn) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 32));
    nt = std::min<int64_t>(nt, n);
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int64_t t = 0; t < nt; ++t) {
        th.emplace_back([&, t]() {
            for (int64_t i = t; i < n; i += nt) fn(i);
        });
    }
    for (auto& x : th) x.join();
}

// Orthonormal associated Legendre functions of order 0 and 1 on [-1, 1]
// (Condon-Shortley phase), Pt_l^m for l = m .. lmax at one point.
// Three-term recurrence in l; no underflow issue for m <= 1.
// Orthonormal associated Legendre functions of orders 0 and 1 at one point,
// by the three-term recurrences in long double (x87 extended precision) and
// rounded once: in double the recurrence loses ~l^2 eps near the poles (4e-11
// relative at l = 2048 on the first ring), in extended precision ~1e-13.
void legendre01(int lmax, long double z, long double sinth, std::vector<double>& p0, std::vector<double>& p1) {
    using LD = long double;
    p0.assign(lmax + 1, 0.0);
    p1.assign(lmax + 1, 0.0);
    LD a0 = std::sqrt(LD(0.5)), a1 = 0;
    p0[0] = double(a0);
    if (lmax >= 1) {
        a1 = std::sqrt(LD(1.5)) * z;
        p0[1] = double(a1);
    }
    for (int l = 2; l <= lmax; ++l) {
        const LD ll = LD(l) * l;
        const LD a = std::sqrt((4 * ll - 1) / ll);
        const LD b = std::sqrt((2 * LD(l) + 1) * (l - 1) * (l - 1) / ((2 * LD(l) - 3) * ll));
        const LD v = a * z * a1 - b * a0;
        a0 = a1;
        a1 = v;
        p0[l] = double(v);
    }
    if (lmax < 1) return;
    LD b0 = -std::sqrt(LD(0.75)) * sinth, b1 = 0;
    p1[1] = double(b0);
    if (lmax >= 2) {
        b1 = std::sqrt(LD(5)) * z * b0;
        p1[2] = double(b1);
    }
    for (int l = 3; l <= lmax; ++l) {
        const LD ll = LD(l) * l;
        const LD a = std::sqrt((4 * ll - 1) / (ll - 1));
        const LD b = std::sqrt((2 * LD(l) + 1) * ((LD(l) - 1) * (l - 1) - 1) / ((2 * LD(l) - 3) * (ll - 1)));
        const LD v = a * z * b1 - b * b0;
        b0 = b1;
        b1 = v;
        p1[l] = double(v);
    }
}

// Householder QR of a column-major m x n matrix (m >= n), in place.
// On return the strictly-lower part holds the reflector vectors (with an
// explicit leading entry stored separately), R is in the upper triangle.
struct QR {
    int64_t m, n;
    std::vector<double> a;     // column-major m x n
    std::vector<double> v0;    // leading entry of each reflector
    std::vector<double> tau;

    void factor() {
        v0.assign(n, 0.0);
        tau.assign(n, 0.0);
        for (int64_t k = 0; k < n; ++k) {
            double* col = &a[k * m];
            double nrm2 = 0.0;
            for (int64_t i = k; i < m; ++i) nrm2 += col[i] * col[i];
            double nrm = std::sqrt(nrm2);
            double x0 = col[k];
            double alpha = (x0 >= 0.0) ? -nrm : nrm;
            double v0k = x0 - alpha;
            // v = (v0k, col[k+1 ..]), tau = 2 / (v^T v)
            double vtv = v0k * v0k + (nrm2 - x0 * x0);
            double t = (vtv > 0.0) ? 2.0 / vtv : 0.0;
            v0[k] = v0k;
            tau[k] = t;
            col[k] = alpha;
            if (t == 0.0) continue;
            parallel_for(n - k - 1, [&](int64_t jj) {
                int64_t j = k + 1 + jj;
                double* cj = &a[j * m];
                double s = v0k * cj[k];
                for (int64_t i = k + 1; i < m; ++i) s += col[i] * cj[i];
                s *= t;
                cj[k] -= s * v0k;
                for (int64_t i = k + 1; i < m; ++i) cj[i] -= s * col[i];
            });
        }
    }

    double r(int64_t i, int64_t j) const { return a[j * m + i]; }

    // Explicit thin Q (m x n, column-major) = H_0 ... H_{n-1} [I; 0].
    std::vector<double> thin_q() const {
        std::vector<double> q(size_t(m) * n, 0.0);
        for (int64_t j = 0; j < n; ++j) q[j * m + j] = 1.0;
        for (int64_t k = n - 1; k >= 0; --k) {
            const double* vk = &a[k * m];
            double v0k = v0[k], t = tau[k];
            if (t == 0.0) continue;
            parallel_for(n - k, [&](int64_t jj) {
                int64_t j = k + jj;
                double* qj = &q[j * m];
                double s = v0k * qj[k];
                for (int64_t i = k + 1; i < m; ++i) s += vk[i] * qj[i];
                s *= t;
                qj[k] -= s * v0k;
                for (int64_t i = k + 1; i < m; ++i) qj[i] -= s * vk[i];
            });
        }
        return q;
    }
};

// Forward complex FFT (e^{-2 pi i jk / M}), M a power of two, FP64.
void host_fft(std::vector<std::complex<double>>& x) {
    const size_t M = x.size();
    for (size_t i = 1, j = 0; i < M; ++i) {
        size_t bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (size_t len = 2; len <= M; len <<= 1) {
        size_t half = len / 2;
        for (size_t st = 0; st < M; st += len) {
            for (size_t k = 0; k < half; ++k) {
                double ang = -2.0 * kPi * double(k) / double(len);
                std::complex<double> w(std::cos(ang), std::sin(ang));
                std::complex<double> u = x[st + k], v = w * x[st + k + half];
                x[st + k] = u + v;
                x[st + k + half] = u - v;
            }
        }
    }
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

int64_t bluestein_length(int64_t L) {
    int64_t M = 1;
    while (M < 2 * L - 1) M <<= 1;
    return M;
}

BlockShape block_shape(int nside, int block) {
    const int p = 2 * nside;
    BlockShape b;
    b.kpar = block >> 1;
    b.sym = block & 1;
    static const int lmins[4] = {0, 1, 1, 2};
    b.lmin = lmins[block];
    b.nl = (p - b.lmin) / 2 + 1;
    b.nk = (b.kpar == 0) ? p / 2 + 1 : p / 2;
    b.nsweep = b.nk - 1;
    return b;
}

RingGeom ring_geom(int nside, int r) {
    RingGeom g;
    const double ns2 = 3.0 * double(nside) * double(nside);
    if (r < nside) {
        const int64_t j = r;
        g.one_minus_z_abs = double(j * j) / ns2;
        g.z = 1.0 - g.one_minus_z_abs;
        g.n = 4 * j;
        g.phi0 = kPi / (4.0 * j);
    } else if (r <= 3 * nside) {
        g.z = 2.0 * double(2 * nside - r) / (3.0 * nside);
        g.one_minus_z_abs = 1.0 - std::fabs(g.z);
        g.n = 4 * int64_t(nside);
        g.phi0 = ((r + 1) % 2) ? kPi / (4.0 * nside) : 0.0;
    } else {
        const int64_t j = 4 * int64_t(nside) - r;
        g.one_minus_z_abs = double(j * j) / ns2;
        g.z = -(1.0 - g.one_minus_z_abs);
        g.n = 4 * j;
        g.phi0 = kPi / (4.0 * j);
    }
    g.start = 0;
    return g;
}

void givens_cs(int l, int mp, double* c, double* s) {
    // s = <Pt_l^mp, Pt_l^{mp-2}> = -sqrt((l-mp+2)(l-mp+1) / ((l+mp)(l+mp-1))),
    // c = sqrt(1 - s^2) with 1 - s^2 formed exactly in integers.
    const int64_t a = int64_t(l - mp + 2) * (l - mp + 1);
    const int64_t d = int64_t(l + mp) * (l + mp - 1);
    const int64_t num_c = d - a;
    *s = -std::sqrt(double(a) / double(d));
    *c = std::sqrt(double(num_c) / double(d));
}

namespace {

void build_uncached(int nside, HostTables& t, bool with_fft) {
    t.nside = nside;
    const int p = 2 * nside;
    t.p = p;
    const int nr = 4 * nside - 1;
    t.rings.resize(nr);
    int64_t start = 0;
    for (int r = 1; r <= nr; ++r) {
        RingGeom g = ring_geom(nside, r);
        g.start = start;
        start += g.n;
        t.rings[r - 1] = g;
    }

    // Pole weights: value at z = 1 of the quadratic through (z_r, mean_r),
    // r = 1, 2, 3 (Lagrange), written with 1 - z for accuracy near the pole.
    {
        double u[3];
        for (int i = 0; i < 3; ++i) {
            const RingGeom& g = t.rings[i];
            u[i] = (g.z >= 0.0) ? g.one_minus_z_abs : 1.0 - g.z;
        }
        for (int i = 0; i < 3; ++i) {
            double w = 1.0;
            for (int j = 0; j < 3; ++j)
                if (j != i) w *= (0.0 - u[j]) / (u[i] - u[j]);
            t.pole_w[i] = w;
        }
    }

    // Half-ring rows h = 0 .. 2 nside: heights and Legendre values.
    const int K = 2 * nside + 1;
    std::vector<std::vector<double>> P0(K), P1(K);
    parallel_for(K, [&](int64_t h) {
        // z and 1 - z of half-ring row h (ring h of the northern hemisphere)
        // from their exact rational forms, in extended precision
        using LD = long double;
        const LD ns = LD(nside);
        LD z, omz;
        if (h == 0) {
            z = 1;
            omz = 0;
        } else if (h < nside) {
            omz = LD(h) * LD(h) / (3 * ns * ns);
            z = 1 - omz;
        } else {
            z = 2 * (2 * ns - LD(h)) / (3 * ns);
            omz = 1 - z;
        }
        const LD sinth = std::sqrt(omz * (2 - omz));
        legendre01(p, z, sinth, P0[h], P1[h]);
    });

    const double s2pi = std::sqrt(2.0 * kPi);
    for (int b = 0; b < 4; ++b) {
        BlockShape bs = block_shape(nside, b);
        // included rows and weights (Sec. 3.2.2 least squares on the doubled
        // grid, reduced to one hemisphere: pole 1, rings 2, equator 1)
        std::vector<int> rows;
        std::vector<double> w;
        for (int h = 0; h < K; ++h) {
            bool pole = (h == 0), eq = (h == 2 * nside);
            if (bs.kpar == 1 && pole) continue;   // order-1 functions vanish at the pole
            if (bs.sym == 1 && eq) continue;      // D- vanishes on the equator
            rows.push_back(h);
            w.push_back((pole || eq) ? 1.0 : 2.0);
        }
        const int64_t m = int64_t(rows.size()), n = bs.nl;
        QR qr;
        qr.m = m;
        qr.n = n;
        qr.a.assign(size_t(m) * n, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            const int l = bs.lmin + 2 * int(j);
            for (int64_t i = 0; i < m; ++i) {
                const double val = (bs.kpar == 0) ? P0[rows[i]][l] : P1[rows[i]][l];
                qr.a[j * m + i] = std::sqrt(w[i]) * val;
            }
        }
        qr.factor();
        std::vector<double> q = qr.thin_q();
        // X = Q R^{-T}: row i solves sum_{k >= j} R[j][k] x_ik = q_ij, j = n-1 .. 0
        std::vector<double>& A = t.ana[b];
        A.assign(size_t(K) * n, 0.0);
        parallel_for(m, [&](int64_t i) {
            std::vector<double> x(n);
            for (int64_t j = n - 1; j >= 0; --j) {
                double s = q[j * m + i];
                for (int64_t k = j + 1; k < n; ++k) s -= qr.r(j, k) * x[k];
                x[j] = s / qr.r(j, j);
            }
            const double f = s2pi * std::sqrt(w[i]);
            for (int64_t j = 0; j < n; ++j) A[size_t(rows[i]) * n + j] = f * x[j];
        });
        // synthesis: E[l'][h] = Pt_l^{kpar}(z_h) / sqrt(2 pi)
        std::vector<double>& E = t.syn[b];
        E.assign(size_t(n) * K, 0.0);
        for (int64_t j = 0; j < n; ++j) {
            const int l = bs.lmin + 2 * int(j);
            for (int h = 0; h < K; ++h) {
                double val = (bs.kpar == 0) ? P0[h][l] : P1[h][l];
                if (bs.sym == 1 && h == 2 * nside) val = 0.0;
                if (bs.kpar == 1 && h == 0) val = 0.0;
                E[size_t(j) * K + h] = val / s2pi;
            }
        }
        // Givens angles, [l'][t-1] pairs
        std::vector<double>& G = t.givens[b];
        const int T = bs.nsweep;
        G.assign(size_t(n) * std::max(T, 1) * 2, 0.0);
        for (int64_t lp = 0; lp < n; ++lp) {
            for (int tt = 1; tt <= T && tt <= lp; ++tt) {
                const int l = bs.lmin + 2 * int(lp);
                const int mp = 2 * tt + bs.kpar;
                double c, s;
                givens_cs(l, mp, &c, &s);
                G[(size_t(lp) * T + (tt - 1)) * 2 + 0] = c;
                G[(size_t(lp) * T + (tt - 1)) * 2 + 1] = s;
            }
        }
    }

    if (!with_fft) return;

    // FFT tables.
    t.fft_max = 4 * nside;
    t.twiddle.assign(size_t(2 * t.fft_max), 0.0);
    for (int i = 0; i < t.fft_max; ++i) {
        const double ang = -2.0 * kPi * double(i) / double(t.fft_max);
        t.twiddle[2 * i] = std::cos(ang);
        t.twiddle[2 * i + 1] = std::sin(ang);
    }
    t.rootoff.assign(nside + 2, 0);
    t.chirpoff.assign(nside + 2, 0);
    t.chirpfftoff.assign(nside + 2, 0);
    t.chirpm.assign(nside + 1, 0);
    int64_t ro = 0, co = 0, fo = 0;
    for (int j = 1; j <= nside; ++j) {
        const int64_t n = 4 * int64_t(j), L = 2 * int64_t(j);
        t.rootoff[j] = ro;
        ro += n + 1;
        t.chirpoff[j] = co;
        t.chirpfftoff[j] = fo;
        if (!is_pow2(L)) {
            const int64_t M = bluestein_length(L);
            t.chirpm[j] = int32_t(M);
            co += L;
            fo += M;
        }
    }
    t.rootoff[nside + 1] = ro;
    t.chirpoff[nside + 1] = co;
    t.chirpfftoff[nside + 1] = fo;
    t.roots.assign(size_t(2 * ro), 0.0);
    t.chirp.assign(size_t(2 * co), 0.0);
    t.chirpfft.assign(size_t(2 * fo), 0.0);
    parallel_for(nside, [&](int64_t jj) {
        const int j = int(jj) + 1;
        const int64_t n = 4 * int64_t(j), L = 2 * int64_t(j);
        double* R = &t.roots[2 * t.rootoff[j]];
        for (int64_t k = 0; k <= n; ++k) {
            // e^{-i pi k / n}; reduce by the exact eighth-turn symmetries is not
            // needed for accuracy at these sizes
            const double ang = -kPi * double(k) / double(n);
            R[2 * k] = std::cos(ang);
            R[2 * k + 1] = std::sin(ang);
        }
        if (t.chirpm[j] == 0) return;
        const int64_t M = t.chirpm[j];
        double* C = &t.chirp[2 * t.chirpoff[j]];
        std::vector<std::complex<double>> bc(M, 0.0);
        for (int64_t k = 0; k < L; ++k) {
            const int64_t e = (k * k) % (2 * L);     // w_k = e^{-i pi k^2 / L}
            const double ang = -kPi * double(e) / double(L);
            C[2 * k] = std::cos(ang);
            C[2 * k + 1] = std::sin(ang);
            std::complex<double> cw(C[2 * k], -C[2 * k + 1]);   // conj(w_k)
            bc[k] = cw;
            if (k > 0) bc[M - k] = cw;
        }
        host_fft(bc);
        double* F = &t.chirpfft[2 * t.chirpfftoff[j]];
        for (int64_t k = 0; k < M; ++k) {
            F[2 * k] = bc[k].real();
            F[2 * k + 1] = bc[k].imag();
        }
    });
}

// ---------------------------------------------------------------------------
// On-disk cache of the tables (HP2SPH_TABLE_CACHE names a directory)
// ---------------------------------------------------------------------------
//
// One file per nside: a header (magic, the build stamp of this file, nside,
// whether the FFT tables are present) and then every table as (count, raw
// bytes).  The build stamp ties a file to the code that wrote it: a rebuilt
// library ignores (and rewrites) files of an earlier build.  Files are
// written to a temporary name and renamed, so a reader never sees a partial
// file; a file that does not parse is rebuilt.

constexpr char kCacheMagic[8] = {'H', 'P', '2', 'S', 'T', 'A', 'B', '1'};
const char* const kBuildStamp = __DATE__ " " __TIME__;

struct CacheFile {
    FILE* f = nullptr;
    ~CacheFile() {
        if (f) std::fclose(f);
    }
};

template <class V>
bool put_vec(FILE* f, const std::vector<V>& v) {
    const uint64_t n = v.size();
    return std::fwrite(&n, sizeof n, 1, f) == 1 && (n == 0 || std::fwrite(v.data(), sizeof(V), n, f) == n);
}

template <class V>
bool get_vec(FILE* f, std::vector<V>& v) {
    uint64_t n = 0;
    if (std::fread(&n, sizeof n, 1, f) != 1 || n > (uint64_t(1) << 36) / sizeof(V)) return false;
    v.resize(n);
    return n == 0 || std::fread(v.data(), sizeof(V), n, f) == n;
}

struct CacheHeader {
    char magic[8];
    char stamp[32];
    int32_t nside, with_fft, fft_max, pad;
    double pole_w[3];
};

bool io_tables(FILE* f, HostTables& t, bool write) {
    auto vec = [&](auto& v) { return write ? put_vec(f, v) : get_vec(f, v); };
    bool ok = vec(t.rings);
    for (int b = 0; b < 4 && ok; ++b) ok = vec(t.ana[b]) && vec(t.syn[b]) && vec(t.givens[b]);
    ok = ok && vec(t.twiddle) && vec(t.rootoff) && vec(t.roots) && vec(t.chirpoff) && vec(t.chirp) &&
         vec(t.chirpfftoff) && vec(t.chirpm) && vec(t.chirpfft);
    return ok;
}

std::string cache_path(const char* dir, int nside) {
    return std::string(dir) + "/hp2sph_tables_nside" + std::to_string(nside) + ".bin";
}

bool cache_load(const char* dir, int nside, bool with_fft, HostTables& t) {
    CacheFile cf;
    cf.f = std::fopen(cache_path(dir, nside).c_str(), "rb");
    if (!cf.f) return false;
    CacheHeader hd{};
    if (std::fread(&hd, sizeof hd, 1, cf.f) != 1) return false;
    if (std::memcmp(hd.magic, kCacheMagic, 8) != 0 || std::strncmp(hd.stamp, kBuildStamp, sizeof hd.stamp) != 0 ||
        hd.nside != nside || (with_fft && !hd.with_fft))
        return false;
    HostTables r;
    if (!io_tables(cf.f, r, false)) return false;
    r.nside = nside;
    r.p = 2 * nside;
    r.fft_max = hd.fft_max;
    for (int i = 0; i < 3; ++i) r.pole_w[i] = hd.pole_w[i];
    if (r.rings.size() != size_t(4 * nside - 1)) return false;
    t = std::move(r);
    return true;
}

void cache_store(const char* dir, int nside, bool with_fft, HostTables& t) {
    const std::string path = cache_path(dir, nside);
    const std::string tmp = path + ".tmp" + std::to_string(long(getpid()));
    bool ok = false;
    {
        CacheFile cf;
        cf.f = std::fopen(tmp.c_str(), "wb");
        if (!cf.f) return;   // an unwritable cache directory only costs the rebuild
        CacheHeader hd{};
        std::memcpy(hd.magic, kCacheMagic, 8);
        std::strncpy(hd.stamp, kBuildStamp, sizeof hd.stamp - 1);
        hd.nside = nside;
        hd.with_fft = with_fft ? 1 : 0;
        hd.fft_max = t.fft_max;
        for (int i = 0; i < 3; ++i) hd.pole_w[i] = t.pole_w[i];
        ok = std::fwrite(&hd, sizeof hd, 1, cf.f) == 1 && io_tables(cf.f, t, true);
        ok = (std::fflush(cf.f) == 0) && ok;
    }
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

}  // namespace

void build_tables(int nside, HostTables& t, bool with_fft) {
    if (nside < 2 || !is_pow2(nside)) throw std::invalid_argument("nside must be a power of two >= 2");
    const char* dir = std::getenv("HP2SPH_TABLE_CACHE");
    if (dir && *dir && cache_load(dir, nside, with_fft, t)) return;
    build_uncached(nside, t, with_fft);
    if (dir && *dir) cache_store(dir, nside, with_fft, t);
}

}  // namespace hp2sph
