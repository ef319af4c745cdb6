// vkt_api.hip -- the C interface of libvkt (include/vkt.h): handles,
// argument validation, the per-thread execution state and kernel dispatch.
//
// The per-thread state mirrors the paper's thread-local ExecutionPolicy
// (Sec. 3.1): the stream work is enqueued on and the arithmetic precision.
// Volumes are device resident; there is no implicit host<->device migration.
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "vkt_internal.h"

namespace {

struct ThreadState {
    hipStream_t stream = nullptr;
    vktPrecision precision = vktPrecisionAuto;
    bool autotune = false;
    bool separable = false;
    bool int8_matrix = false;
    int64_t row_pair_min_cells = int64_t(1) << 24;
    bool init = false;
};
thread_local ThreadState t_state;

ThreadState& state()
{
    if (!t_state.init) {
        t_state.init = true;
        if (const char* p = std::getenv("VKT_PRECISION")) {
            if (!std::strcmp(p, "fp32")) t_state.precision = vktPrecisionFP32;
            else if (!std::strcmp(p, "splitbf16")) t_state.precision = vktPrecisionSplitBF16;
            else if (!std::strcmp(p, "splitbf16x6")) t_state.precision = vktPrecisionSplitBF16x6;
        }
        if (const char* p = std::getenv("VKT_AUTOTUNE")) t_state.autotune = p[0] == '1';
        if (const char* p = std::getenv("VKT_SEPARABLE")) t_state.separable = p[0] == '1';
        if (const char* p = std::getenv("VKT_INT8_MATRIX")) t_state.int8_matrix = p[0] == '1';
        if (const char* p = std::getenv("VKT_ROW_PAIR_MIN_CELLS")) {
            char* end = nullptr;
            const long long v = std::strtoll(p, &end, 10);
            if (end != p && v >= 0) t_state.row_pair_min_cells = v;
        }
    }
    return t_state;
}

// Live handles, so that stale or foreign handles are rejected instead of
// dereferenced.
std::mutex g_mu;
std::unordered_set<const void*> g_volumes, g_filters;
uint64_t g_filter_serial = 0;

using vkt::from_hip;
using vkt::live_filter;
using vkt::live_volume;

bool valid_format(int f) { return f >= vktDataFormatUInt8 && f <= vktDataFormatFloat32; }

int64_t cells(const vktStructuredVolume_* v)
{
    return (int64_t)v->dims[0] * v->dims[1] * v->dims[2];
}

// Raw stored value for Fill: integer formats map [lo, hi] onto [0, max] with
// half-up rounding and saturation; Float32 stores the value.
uint32_t raw_fill_bits(const vktStructuredVolume_* v, float value)
{
    if (v->fmt == vktDataFormatFloat32) {
        uint32_t u;
        std::memcpy(&u, &value, 4);
        return u;
    }
    const double mx = v->fmt == vktDataFormatUInt8 ? 255.0 : 65535.0;
    double r = std::floor(((double)value - v->lo) / ((double)v->hi - v->lo) * mx + 0.5);
    if (!(r >= 0.0)) r = 0.0;  // also maps NaN to 0
    if (r > mx) r = mx;
    return (uint32_t)r;
}

vktError create_volume(vktStructuredVolume* out, int32_t dx, int32_t dy, int32_t dz,
                       vktDataFormat f, void* dev, bool own, const float cell[3],
                       float lo, float hi)
{
    if (!out || dx <= 0 || dy <= 0 || dz <= 0 || !valid_format(f)) return vktInvalidValue;
    if (f != vktDataFormatFloat32 && !(lo != hi)) return vktInvalidValue;
    const int64_t n = (int64_t)dx * dy * dz;
    const size_t bytes = (size_t)n * vkt::cell_bytes(f);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return vktDeviceError;
    if (own) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return from_hip(e);
        e = hipMemsetAsync(p, 0, bytes, state().stream);
        if (e != hipSuccess) { (void)hipFree(p); return from_hip(e); }
        dev = p;
    }
    auto* v = new (std::nothrow) vktStructuredVolume_{{dx, dy, dz}, f,
                                                      {cell[0], cell[1], cell[2]},
                                                      lo, hi, dev, own, device};
    if (!v) {
        if (own) (void)hipFree(dev);
        return vktOutOfMemory;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_volumes.insert(v);
    }
    *out = v;
    return vktNoError;
}

// Rank-1 test of a k^3 filter (index a + k (b + k c)), pivot p at the
// largest |w| (a*, b*, c*).  The rows through the pivot, w[c*][b*][:],
// w[c*][:][a*] and w[:][b*][a*], are proportional to the factors.
//  * Integer filters: each row divided by the gcd of its entries gives a
//    primitive integer vector x, y, z (sign: positive at the pivot); then
//    w = alpha x (x) y (x) z with alpha = p / (x[a*] y[b*] z[c*]) an integer,
//    and u = alpha x, v = y, t = z reproduce w exactly (checked exactly, so
//    sum|u| sum|v| sum|t| = sum|w|).
//  * Float filters: u = w[c*][b*][:], v = w[c*][:][a*] / p,
//    t = w[:][b*][a*] / p, accepted when every weight is reproduced to
//    within 2^-20 of itself (plus 2^-149, the FP32 underflow step): FP32
//    weights that are roundings of an exact outer product satisfy this (each
//    product of three weights over the pivot squared carries at most about
//    6 roundings of 2^-24), and a per-weight relative bound keeps the three
//    passes within 2^-20 sum|w||s| of the dense sum for every volume -- a
//    bound on the largest or the summed deviation would not (weights near
//    zero where the cells are large).
struct Rank1 {
    bool ok = false;
    std::vector<double> u, v, t;
};
int64_t gcd64(int64_t a, int64_t b)
{
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const int64_t r = a % b;
        a = b;
        b = r;
    }
    return a;
}
Rank1 rank1(int k, const std::vector<double>& w, bool exact_int)
{
    Rank1 r;
    const int n = k * k * k;
    int ip = 0;
    for (int i = 1; i < n; ++i)
        if (std::fabs(w[i]) > std::fabs(w[ip])) ip = i;
    const double p = w[ip];
    if (p == 0.0) return r;
    const int as = ip % k, bs = (ip / k) % k, cs = ip / (k * k);
    auto at = [&](int a, int b, int c) { return w[a + k * (b + k * c)]; };
    std::vector<double> ru(k), rv(k), rt(k);
    for (int i = 0; i < k; ++i) {
        ru[i] = at(i, bs, cs);
        rv[i] = at(as, i, cs);
        rt[i] = at(as, bs, i);
    }
    if (exact_int) {
        std::vector<int64_t> x(k), y(k), z(k);
        auto primitive = [&](const std::vector<double>& row, int piv, std::vector<int64_t>& out) {
            int64_t g = 0;
            for (int i = 0; i < k; ++i) g = gcd64(g, (int64_t)row[i]);
            const int64_t s = row[piv] < 0 ? -g : g;
            for (int i = 0; i < k; ++i) out[i] = (int64_t)row[i] / s;
        };
        primitive(ru, as, x);
        primitive(rv, bs, y);
        primitive(rt, cs, z);
        const int64_t den = x[as] * y[bs] * z[cs];  // > 0, divides p for rank 1
        if (den == 0 || (int64_t)p % den != 0) return r;
        const int64_t alpha = (int64_t)p / den;
        for (int c = 0; c < k; ++c)
            for (int b = 0; b < k; ++b)
                for (int a = 0; a < k; ++a) {
                    const __int128 prod = (__int128)(alpha * x[a]) * y[b] * z[c];
                    if (prod != (__int128)(int64_t)at(a, b, c)) return r;
                }
        r.u.resize(k);
        r.v.resize(k);
        r.t.resize(k);
        for (int i = 0; i < k; ++i) {
            r.u[i] = (double)(alpha * x[i]);
            r.v[i] = (double)y[i];
            r.t[i] = (double)z[i];
        }
    } else {
        r.u = ru;
        r.v = rv;
        r.t = rt;
        for (int i = 0; i < k; ++i) {
            r.v[i] /= p;
            r.t[i] /= p;
        }
        for (int c = 0; c < k; ++c)
            for (int b = 0; b < k; ++b)
                for (int a = 0; a < k; ++a) {
                    const double wv = at(a, b, c);
                    if (std::fabs(r.u[a] * r.v[b] * r.t[c] - wv) >
                        std::ldexp(std::fabs(wv), -20) + std::ldexp(1.0, -149))
                        return r;
                }
    }
    r.ok = true;
    return r;
}

vktError create_filter(vktFilter* out, int32_t k, const float* wf, const int32_t* wi,
                       int32_t divisor)
{
    if (!out || (!wf && !wi) || k < 1 || k > 15 || (k % 2) == 0) return vktInvalidValue;
    const int n = k * k * k;
    std::vector<float> hf(n);
    std::vector<int32_t> hi;
    int64_t sum_abs = 0;
    if (wi) {
        if (divisor < 1 || divisor > (1 << 29)) return vktInvalidValue;
        hi.assign(wi, wi + n);
        for (int i = 0; i < n; ++i) {
            if (hi[i] <= -(1 << 23) || hi[i] >= (1 << 23)) return vktInvalidValue;
            sum_abs += hi[i] < 0 ? -(int64_t)hi[i] : hi[i];
            hf[i] = (float)hi[i];  // exact below 2^24
        }
    } else {
        std::memcpy(hf.data(), wf, n * sizeof(float));
    }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return vktDeviceError;
    float* dwf = nullptr;
    int32_t* dwi = nullptr;
    // zero-padded copies (wide scalar loads of the last weight group)
    const size_t npad = (size_t)n + vkt::kWeightPad;
    hf.resize(npad, 0.f);
    hipError_t e = hipMalloc(&dwf, npad * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(dwf, hf.data(), npad * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess && wi) {
        hi.resize(npad, 0);
        e = hipMalloc(&dwi, npad * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(dwi, hi.data(), npad * sizeof(int32_t), hipMemcpyHostToDevice);
    }
    // 8-bit packed rows for the dot-product path (uint8 volumes): weights all
    // in [0, 255] (unsigned) or all in [-128, 127] (signed), k <= 7, and
    // sum|w| and D small enough for its exact FP32 epilogue
    uint32_t* dwq = nullptr;
    bool q_ok = false, q_signed = false;
    int64_t sum_int = 0;
    if (wi) {
        bool u8 = true, s8 = true;
        for (int i = 0; i < n; ++i) {
            u8 = u8 && hi[i] >= 0 && hi[i] <= 255;
            s8 = s8 && hi[i] >= -128 && hi[i] <= 127;
            sum_int += hi[i];
        }
        q_ok = (k == 3 || k == 5 || k == 7) && (u8 || s8) && sum_abs <= 2048 &&
               divisor <= (1 << 19);
        q_signed = !u8;
    }
    if (e == hipSuccess && q_ok) {
        const int nh = (k + 3) / 4, nw = vkt::dot4_words(k);
        std::vector<uint32_t> hq((size_t)nw + vkt::kWeightPad, 0u);
        for (int row = 0; row < k * k; ++row)
            for (int a = 0; a < k; ++a)
                hq[(size_t)row * nh + a / 4] |= ((uint32_t)hi[(size_t)row * k + a] & 0xffu)
                                                << (8 * (a % 4));
        e = hipMalloc(&dwq, hq.size() * sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemcpy(dwq, hq.data(), hq.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    }
    // int8 matrix-core operands (k = 3, signed 8-bit weights, the same bounds
    // as the dot products): for filter plane c and lane l (m = l mod 16,
    // K chunk g = l / 16), byte i of W_c pairs with byte i of the lane's
    // staged-cell chunk: g < 3 holds input row b = g, columns x0t + i, so the
    // tap is a = i - m + 1; chunk 3 holds the cells left (byte 2b, tap 0 of
    // output m = 0) and right (byte 2b + 1, tap 2 of m = 15) of row b
    uint32_t* dwm = nullptr;
    bool m8_ok = false;
    if (e == hipSuccess && wi && k == 3 && sum_abs <= 2048 && divisor <= (1 << 19)) {
        m8_ok = true;
        for (int i = 0; i < n; ++i) m8_ok = m8_ok && hi[i] >= -128 && hi[i] <= 127;
    }
    if (e == hipSuccess && m8_ok) {
        std::vector<uint8_t> hm(vkt::kI8mmaTableBytes, 0);
        auto wk = [&](int c, int b, int a) { return (uint8_t)(int8_t)hi[(size_t)a + 3 * (b + 3 * c)]; };
        for (int c = 0; c < 3; ++c)
            for (int l = 0; l < 64; ++l) {
                const int m = l % 16, g = l / 16;
                uint8_t* row = &hm[(size_t)(c * 64 + l) * 16];
                if (g < 3) {
                    for (int i = 0; i < 16; ++i) {
                        const int a = i - m + 1;
                        if (a >= 0 && a < 3) row[i] = wk(c, g, a);
                    }
                } else {
                    for (int b = 0; b < 3; ++b) {
                        if (m == 0) row[2 * b] = wk(c, b, 0);
                        if (m == 15) row[2 * b + 1] = wk(c, b, 2);
                    }
                }
            }
        e = hipMalloc(&dwm, hm.size());
        if (e == hipSuccess) e = hipMemcpy(dwm, hm.data(), hm.size(), hipMemcpyHostToDevice);
    }
    // rank-1 factors for the separable path
    float* dsep = nullptr;
    Rank1 r1;
    int64_t sep_sum_abs = 0;
    if (e == hipSuccess) {
        std::vector<double> wd(n);
        for (int i = 0; i < n; ++i) wd[i] = wi ? (double)hi[i] : (double)hf[i];
        r1 = rank1(k, wd, wi != nullptr);
    }
    if (e == hipSuccess && r1.ok) {
        std::vector<float> hs(3 * 16 + vkt::kWeightPad, 0.f);
        double su = 0, sv = 0, st = 0;
        for (int i = 0; i < k; ++i) {
            hs[i] = (float)r1.u[i];
            hs[16 + i] = (float)r1.v[i];
            hs[32 + i] = (float)r1.t[i];
            su += std::fabs(r1.u[i]);
            sv += std::fabs(r1.v[i]);
            st += std::fabs(r1.t[i]);
        }
        const double prod = su * sv * st;
        sep_sum_abs = prod < 9.0e18 ? (int64_t)prod : INT64_MAX;
        e = hipMalloc(&dsep, hs.size() * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(dsep, hs.data(), hs.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        if (dwf) (void)hipFree(dwf);
        if (dwi) (void)hipFree(dwi);
        if (dwq) (void)hipFree(dwq);
        if (dwm) (void)hipFree(dwm);
        if (dsep) (void)hipFree(dsep);
        return from_hip(e);
    }
    // power-of-two weight scale for fp16 operand splitting
    float amax = 0.f;
    for (int i = 0; i < n; ++i) amax = std::fmax(amax, std::fabs(hf[i]));
    float wscale = 1.f;
    if (amax > 0.f && std::isfinite(amax)) {
        int ex = 0;
        std::frexp(amax, &ex);                 // amax in [2^(ex-1), 2^ex)
        wscale = std::ldexp(1.f, 15 - ex);     // amax * wscale in [2^14, 2^15)
    }
    auto* f = new (std::nothrow) vktFilter_{k, wi != nullptr, wi ? divisor : 1, sum_abs,
                                            wscale, 0, dwf, dwi, dwq, q_ok, q_signed,
                                            sum_int, m8_ok, dwm, r1.ok, sep_sum_abs, dsep,
                                            device};
    if (!f) {
        (void)hipFree(dwf);
        if (dwi) (void)hipFree(dwi);
        if (dwq) (void)hipFree(dwq);
        if (dwm) (void)hipFree(dwm);
        if (dsep) (void)hipFree(dsep);
        return vktOutOfMemory;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        f->serial = ++g_filter_serial;
        g_filters.insert(f);
    }
    *out = f;
    return vktNoError;
}

}  // namespace

namespace vkt {

bool live_volume(const vktStructuredVolume_* v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return v && g_volumes.count(v);
}

bool live_filter(const vktFilter_* f)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return f && g_filters.count(f);
}

vktError from_hip(hipError_t e)
{
    if (e == hipSuccess) return vktNoError;
    if (e == hipErrorOutOfMemory) return vktOutOfMemory;
    return vktDeviceError;
}

hipStream_t thread_stream() { return state().stream; }
vktPrecision thread_precision() { return state().precision; }
bool thread_autotune() { return state().autotune; }
bool thread_separable() { return state().separable; }
bool thread_int8_matrix() { return state().int8_matrix; }
int64_t thread_row_pair_min_cells() { return state().row_pair_min_cells; }

VolDesc make_desc(const FilterJob& j, int tz, ClassGeom g)
{
    VolDesc a{};
    a.src = j.src;
    a.dst = j.dst;
    a.X = j.X;
    a.Y = j.Y;
    a.Z = j.Z;
    a.mode = j.mode;
    a.tz = tz;
    a.rx0 = j.roi[0];
    a.ry0 = j.roi[1];
    a.rz0 = j.roi[2];
    a.rx1 = j.roi[3];
    a.ry1 = j.roi[4];
    a.rz1 = j.roi[5];
    a.tiles_x = (a.rx1 - a.rx0 + g.tx - 1) / g.tx;
    a.tiles_y = (a.ry1 - a.ry0 + g.ty - 1) / g.ty;
    a.woff = 0;
    if (j.fmt == vktDataFormatFloat32) a.epi = j.int_filter ? kEpiFloatDiv : kEpiFloat;
    else a.epi = j.int_filter ? kEpiIntDiv : kEpiRound;
    a.D = j.D;
    a.div2D = j.div2D;
    a.inv_D = j.inv_D;
    a.vec_ok = j.vec_store ? 1 : 0;
    a.wscale = j.fmt == vktDataFormatFloat32 ? 1.0f : j.wscale;  // bf16 pieces are unscaled
    a.unscale = 1.0f / a.wscale;
    a.bias = j.q_bias;
    return a;
}

vktError build_job(const vktStructuredVolume_* dst, const vktStructuredVolume_* src,
                   const vktFilter_* filt, int mode, vktPrecision prec, FilterJob& j,
                   bool& mfma, bool& six, const int32_t* roi, bool allow_sep)
{
    if (!live_volume(dst) || !live_volume(src) || !live_filter(filt)) return vktInvalidValue;
    if (mode < vktAddressModeClamp || mode > vktAddressModeBorder) return vktInvalidValue;
    if (dst->fmt != src->fmt) return vktInvalidValue;
    for (int a = 0; a < 3; ++a)
        if (dst->dims[a] != src->dims[a]) return vktInvalidValue;
    const int64_t bytes = cells(src) * cell_bytes(src->fmt);
    const char* d0 = static_cast<const char*>(dst->dev);
    const char* s0 = static_cast<const char*>(src->dev);
    if (d0 < s0 + bytes && s0 < d0 + bytes) return vktInvalidValue;  // overlap
    // in-plane byte offsets are 32-bit in the kernels
    if ((int64_t)src->dims[0] * src->dims[1] * cell_bytes(src->fmt) >= (int64_t(1) << 31))
        return vktUnsupported;

    j = FilterJob{};
    j.src = src->dev;
    j.dst = dst->dev;
    j.X = src->dims[0];
    j.Y = src->dims[1];
    j.Z = src->dims[2];
    const int32_t whole[6] = {0, 0, 0, j.X, j.Y, j.Z};
    std::memcpy(j.roi, roi ? roi : whole, sizeof(j.roi));
    j.mode = mode;
    j.fmt = src->fmt;
    j.k = filt->k;
    j.wf = filt->d_wf;
    j.wi = filt->d_wi;
    j.int_filter = filt->is_int;
    j.D = filt->divisor;
    j.inv_D = 1.0f / (float)filt->divisor;
    j.int_acc = false;
    if (filt->is_int && src->fmt != vktDataFormatFloat32) {
        const int64_t mx = src->fmt == vktDataFormatUInt8 ? 255 : 65535;
        if (filt->sum_abs_int * mx > (int64_t(1) << 30)) return vktUnsupported;
        // FP32 sums of integer products are exact while |partial sums| < 2^24;
        // beyond that the kernel accumulates in int32.
        j.int_acc = filt->sum_abs_int * mx >= (int64_t(1) << 24);
        j.div2D = make_udiv(2u * (uint32_t)filt->divisor);
    }
    // 4-cell vector stores: rows, the region's first column and the buffer
    // 4-cell aligned
    j.vec_store = (j.X % 4 == 0) && (j.roi[0] % 4 == 0) &&
                  (reinterpret_cast<uintptr_t>(dst->dev) % (4 * cell_bytes(src->fmt)) == 0);
    j.wscale = filt->wscale;
    // Plan: float-weight filters with k >= 5 run on the matrix cores unless
    // the precision is FP32; everything else (k < 5, integer weights, whose
    // results are exact integers) runs on the vector ALUs, uint8 volumes with
    // small integer weights as 8-bit dot products (4-byte rows and buffers).
    mfma = !filt->is_int && filt->k >= 5 && prec != vktPrecisionFP32;
    j.dot4 = filt->q_ok && src->fmt == vktDataFormatUInt8 && j.X % 4 == 0 &&
             j.roi[0] % 4 == 0 && j.roi[3] % 4 == 0 &&
             reinterpret_cast<uintptr_t>(src->dev) % 4 == 0 &&
             reinterpret_cast<uintptr_t>(dst->dev) % 4 == 0;
    j.q_signed = filt->q_signed;
    j.wq = filt->d_wq;
    // Rank-1 filters on the separable path when the thread asks for it.  For
    // integer filters on integer cells the three passes must stay exact in
    // FP32: every partial sum an integer below 2^24.
    j.sep = false;
    j.wsep = filt->d_sep;
    if (allow_sep && state().separable && filt->sep_ok) {
        if (!filt->is_int) {
            j.sep = true;
        } else {
            const int64_t mx = src->fmt == vktDataFormatUInt8 ? 255 : 65535;
            j.sep = src->fmt == vktDataFormatFloat32 ||
                    filt->sep_sum_abs * mx < (int64_t(1) << 24);
        }
        // (k = 3 integer filters on uint8 stay on the 8-bit dot products:
        // measured faster than the three passes there)
        if (j.dot4 && filt->k <= 3) j.sep = false;
        if (j.sep) {
            mfma = false;
            j.dot4 = false;
        }
    }
    if (j.dot4) {
        // floor(T/D + 1/2) as round-to-nearest(T * (1/D) + bias); signed
        // weights add the 128 * sum(w) the cells lost by entering as s - 128
        const double D = (double)filt->divisor;
        j.q_bias = (float)(0.25 / D + (filt->q_signed ? 128.0 * (double)filt->sum_int / D : 0.0));
        // k = 3 with signed 8-bit weights: exact int8 products on the matrix
        // cores (cells always enter as s - 128) when the thread enables them
        j.i8mma = filt->m8_ok && state().int8_matrix;
        j.wm = filt->d_wm;
        j.m8_bias = (float)(0.25 / D + 128.0 * (double)filt->sum_int / D);
    }
    // float32 cells: the 6-product split keeps every product term down to
    // 2^-16 relative (about 1e-7 after rounding); Auto uses it.  The 3-product
    // split drops three terms of up to 2^-16 each and is opt-in.
    six = prec == vktPrecisionSplitBF16x6 || prec == vktPrecisionAuto;
    return vktNoError;
}

// k = 5, 7 run on 32x32x16 tiles over row pairs, except where the 16x16x32
// kernel measured faster: uint8 / uint16 and 6-product float32 with k = 7 on
// 512^3 volumes, and output regions of at most the thread's row-pair
// threshold (default 2^24 cells: 256 uneven uint16 volumes of up to 256^3 in
// one batch take 2.59 ms with the 16x16x32 kernel's 16-row tiles against
// 2.81 ms with row pairs for k = 5).  Single and batched launches choose
// alike, so a batch reproduces its volumes' single launches bit for bit.
bool mfma_row_pairs(const FilterJob& j, bool six_products)
{
    const int64_t cells =
        (int64_t)(j.roi[3] - j.roi[0]) * (j.roi[4] - j.roi[1]) * (j.roi[5] - j.roi[2]);
    return (j.k == 5 || (j.k == 7 && j.fmt == vktDataFormatFloat32 && !six_products)) &&
           cells > state().row_pair_min_cells;
}

hipError_t launch_filter_mfma(const FilterJob& j, bool six_products, hipStream_t s)
{
    if (j.k >= 9) return launch_filter_mfma_s32(j, six_products, s);
    return mfma_row_pairs(j, six_products) ? launch_filter_mfma_rp(j, six_products, s)
                                           : launch_filter_mfma_s16(j, six_products, s);
}

const void* mfma_batched_kernel(vktDataFormat f, int k, bool six_products, bool row_pairs,
                                int variant)
{
    if (k >= 9) return mfma_batched_kernel_s32(f, k, six_products, variant);
    return row_pairs ? mfma_batched_kernel_rp(f, k, six_products)
                     : mfma_batched_kernel_s16(f, k, six_products, variant);
}

ClassGeom mfma_geom(vktDataFormat f, int k, bool six_products, bool row_pairs, int variant)
{
    if (k >= 9) return mfma_geom_s32(f, k, six_products, variant);
    return row_pairs ? mfma_geom_rp(f, k, six_products)
                     : mfma_geom_s16(f, k, six_products, variant);
}

int resident_wgs(const void* func)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({func, dev});
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 1;
    const int n = per_cu * cus;
    cache[{func, dev}] = n;
    return n;
}

int plan_tz(int64_t ntiles, int Z, int k, int tz_min, int tz_max, int slots, int mod)
{
    if (Z <= tz_min) return Z;
    if (tz_max > Z) tz_max = Z;
    if (tz_max < tz_min) tz_max = tz_min;
    int best = tz_max;
    double best_cost = -1.0;
    for (int tz = tz_min; tz <= tz_max; ++tz) {
        if (mod > 1 && tz % mod != 1 % mod && tz != Z) continue;
        const int64_t nwg = ntiles * ((Z + tz - 1) / tz);
        const int64_t rounds = (nwg + slots - 1) / slots;
        const double cost = (double)rounds * (tz + k - 1);
        if (best_cost < 0.0 || cost < best_cost) {  // ties keep the smaller tz
            best_cost = cost;
            best = tz;
        }
    }
    return best;
}

UDiv make_udiv(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;  // l = ceil(log2 d)
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    UDiv r;
    r.m = (uint32_t)m;
    r.sh1 = l < 1 ? l : 1;
    r.sh2 = l > 1 ? l - 1 : 0;
    return r;
}

}  // namespace vkt

extern "C" {

vktError vktStructuredVolumeCreate(vktStructuredVolume* volume, int32_t dimX,
                                   int32_t dimY, int32_t dimZ, vktDataFormat format,
                                   float cellX, float cellY, float cellZ, float lo,
                                   float hi)
{
    const float cell[3] = {cellX, cellY, cellZ};
    return create_volume(volume, dimX, dimY, dimZ, format, nullptr, true, cell, lo, hi);
}

vktError vktStructuredVolumeCreateFromDevicePtr(vktStructuredVolume* volume, int32_t dimX,
                                                int32_t dimY, int32_t dimZ,
                                                vktDataFormat format, void* devPtr,
                                                float lo, float hi)
{
    if (!devPtr || !valid_format(format)) return vktInvalidValue;
    if (reinterpret_cast<uintptr_t>(devPtr) % vkt::cell_bytes(format)) return vktInvalidValue;
    const float cell[3] = {1.f, 1.f, 1.f};
    return create_volume(volume, dimX, dimY, dimZ, format, devPtr, false, cell, lo, hi);
}

vktError vktStructuredVolumeDestroy(vktStructuredVolume v)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!v || !g_volumes.erase(v)) return vktInvalidValue;
    }
    hipError_t e = hipSuccess;
    if (v->owned) e = hipFree(v->dev);
    delete v;
    return from_hip(e);
}

vktError vktStructuredVolumeGetDevicePtr(vktStructuredVolume v, void** p)
{
    if (!live_volume(v) || !p) return vktInvalidValue;
    *p = v->dev;
    return vktNoError;
}

vktError vktStructuredVolumeGetDims(vktStructuredVolume v, int32_t* dx, int32_t* dy,
                                    int32_t* dz)
{
    if (!live_volume(v) || !dx || !dy || !dz) return vktInvalidValue;
    *dx = v->dims[0];
    *dy = v->dims[1];
    *dz = v->dims[2];
    return vktNoError;
}

vktError vktStructuredVolumeGetDataFormat(vktStructuredVolume v, vktDataFormat* f)
{
    if (!live_volume(v) || !f) return vktInvalidValue;
    *f = v->fmt;
    return vktNoError;
}

vktError vktFilterCreate(vktFilter* filter, int32_t k, const float* weights)
{
    if (!weights) return vktInvalidValue;
    return create_filter(filter, k, weights, nullptr, 1);
}

vktError vktFilterCreateInt(vktFilter* filter, int32_t k, const int32_t* weights,
                            int32_t divisor)
{
    if (!weights) return vktInvalidValue;
    return create_filter(filter, k, nullptr, weights, divisor);
}

vktError vktFilterDestroy(vktFilter f)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!f || !g_filters.erase(f)) return vktInvalidValue;
    }
    hipError_t e = hipFree(f->d_wf);
    for (void* p : {(void*)f->d_wi, (void*)f->d_wq, (void*)f->d_wm, (void*)f->d_sep}) {
        if (!p) continue;
        hipError_t e2 = hipFree(p);
        if (e == hipSuccess) e = e2;
    }
    delete f;
    return from_hip(e);
}

vktError vktFill(vktStructuredVolume v, float value)
{
    if (!live_volume(v)) return vktInvalidValue;
    return from_hip(vkt::launch_fill(v->dev, vkt::cell_bytes(v->fmt), cells(v),
                                     raw_fill_bits(v, value), state().stream));
}

vktError vktFillRange(vktStructuredVolume v, int32_t x0, int32_t y0, int32_t z0,
                      int32_t x1, int32_t y1, int32_t z1, float value)
{
    if (!live_volume(v)) return vktInvalidValue;
    const int32_t first[3] = {x0, y0, z0}, last[3] = {x1, y1, z1};
    for (int a = 0; a < 3; ++a)
        if (first[a] < 0 || last[a] > v->dims[a] || first[a] > last[a]) return vktInvalidValue;
    return from_hip(vkt::launch_fill_range(v->dev, vkt::cell_bytes(v->fmt), v->dims[0],
                                           v->dims[1], first, last, raw_fill_bits(v, value),
                                           state().stream));
}

vktError vktFillSV(vktStructuredVolume v, float value) { return vktFill(v, value); }

vktError vktFillRangeSV(vktStructuredVolume v, int32_t x0, int32_t y0, int32_t z0,
                        int32_t x1, int32_t y1, int32_t z1, float value)
{
    return vktFillRange(v, x0, y0, z0, x1, y1, z1, value);
}

vktError vktApplyFilter(vktStructuredVolume dst, vktStructuredVolume src, vktFilter filt,
                        vktAddressMode mode)
{
    vkt::FilterJob j;
    bool mfma = false, six = false;
    const vktError e = vkt::build_job(dst, src, filt, mode, state().precision, j, mfma, six);
    if (e != vktNoError) return e;
    if (j.sep) return from_hip(vkt::launch_filter_sep(j, state().stream));
    if (mfma) return from_hip(vkt::launch_filter_mfma(j, six, state().stream));
    if (j.i8mma) return from_hip(vkt::launch_filter_i8mma(j, state().stream));
    if (j.dot4) return from_hip(vkt::launch_filter_dot4(j, state().stream));
    return from_hip(vkt::launch_filter_valu(j, state().stream));
}

vktError vktApplyFilterRange(vktStructuredVolume dst, vktStructuredVolume src, vktFilter filt,
                             int32_t x0, int32_t y0, int32_t z0, int32_t x1, int32_t y1,
                             int32_t z1, vktAddressMode mode)
{
    if (!vkt::live_volume(src)) return vktInvalidValue;
    const int32_t roi[6] = {x0, y0, z0, x1, y1, z1};
    for (int a = 0; a < 3; ++a)
        if (roi[a] < 0 || roi[a] > roi[a + 3] || roi[a + 3] > src->dims[a]) return vktInvalidValue;
    vkt::FilterJob j;
    bool mfma = false, six = false;
    const vktError e =
        vkt::build_job(dst, src, filt, mode, state().precision, j, mfma, six, roi);
    if (e != vktNoError) return e;
    if (x0 == x1 || y0 == y1 || z0 == z1) return vktNoError;  // empty region
    if (j.sep) return from_hip(vkt::launch_filter_sep(j, state().stream));
    if (mfma) return from_hip(vkt::launch_filter_mfma(j, six, state().stream));
    if (j.i8mma) return from_hip(vkt::launch_filter_i8mma(j, state().stream));
    if (j.dot4) return from_hip(vkt::launch_filter_dot4(j, state().stream));
    return from_hip(vkt::launch_filter_valu(j, state().stream));
}

vktError vktResample(vktStructuredVolume dst, vktStructuredVolume src)
{
    if (!live_volume(dst) || !live_volume(src) || dst->fmt != src->fmt) return vktInvalidValue;
    const int64_t sb = cells(src) * vkt::cell_bytes(src->fmt);
    const int64_t db = cells(dst) * vkt::cell_bytes(dst->fmt);
    const char* d0 = static_cast<const char*>(dst->dev);
    const char* s0 = static_cast<const char*>(src->dev);
    if (d0 < s0 + sb && s0 < d0 + db) return vktInvalidValue;  // overlap
    return from_hip(vkt::launch_resample(src->dev, dst->dev, src->fmt, src->dims, dst->dims,
                                         state().stream));
}

vktError vktFlip(vktStructuredVolume dst, vktStructuredVolume src, vktAxis axis)
{
    if (!live_volume(dst) || !live_volume(src) || dst->fmt != src->fmt) return vktInvalidValue;
    if ((int)axis < vktAxisX || (int)axis > vktAxisZ) return vktInvalidValue;
    for (int a = 0; a < 3; ++a)
        if (dst->dims[a] != src->dims[a]) return vktInvalidValue;
    const int64_t bytes = cells(src) * vkt::cell_bytes(src->fmt);
    const char* d0 = static_cast<const char*>(dst->dev);
    const char* s0 = static_cast<const char*>(src->dev);
    if (d0 != s0 && d0 < s0 + bytes && s0 < d0 + bytes) return vktInvalidValue;  // partial overlap
    return from_hip(vkt::launch_flip(src->dev, dst->dev, src->fmt, src->dims, (int)axis,
                                     state().stream));
}

vktError vktResampleSV(vktStructuredVolume dst, vktStructuredVolume src)
{
    return vktResample(dst, src);
}

vktError vktFlipSV(vktStructuredVolume dst, vktStructuredVolume src, vktAxis axis)
{
    return vktFlip(dst, src, axis);
}

vktError vktSetSeparable(int enable)
{
    state().separable = enable != 0;
    return vktNoError;
}

vktError vktGetSeparable(int* enable)
{
    if (!enable) return vktInvalidValue;
    *enable = state().separable ? 1 : 0;
    return vktNoError;
}

vktError vktSetInt8Matrix(int enable)
{
    state().int8_matrix = enable != 0;
    return vktNoError;
}

vktError vktGetInt8Matrix(int* enable)
{
    if (!enable) return vktInvalidValue;
    *enable = state().int8_matrix ? 1 : 0;
    return vktNoError;
}

vktError vktSetRowPairMinCells(int64_t cells)
{
    if (cells < 0) return vktInvalidValue;
    state().row_pair_min_cells = cells;
    return vktNoError;
}

vktError vktGetRowPairMinCells(int64_t* cells)
{
    if (!cells) return vktInvalidValue;
    *cells = state().row_pair_min_cells;
    return vktNoError;
}

vktError vktFilterIsSeparable(vktFilter filter, int* separable)
{
    if (!separable || !vkt::live_filter(filter)) return vktInvalidValue;
    *separable = filter->sep_ok ? 1 : 0;
    return vktNoError;
}

vktError vktGetFilterPath(vktStructuredVolume dst, vktStructuredVolume src, vktFilter filt,
                          vktAddressMode mode, vktFilterPath* path, int32_t* products)
{
    if (!path) return vktInvalidValue;
    vkt::FilterJob j;
    bool mfma = false, six = false;
    const vktError e = vkt::build_job(dst, src, filt, mode, state().precision, j, mfma, six);
    if (e != vktNoError) return e;
    int32_t p = 1;
    if (j.sep) *path = vktFilterPathSeparable;
    else if (mfma) {
        *path = vktFilterPathSplitMatrix;
        p = j.fmt == vktDataFormatUInt8 ? 2 : (j.fmt == vktDataFormatUInt16 ? 4 : (six ? 6 : 3));
    } else if (j.i8mma) *path = vktFilterPathInt8Matrix;
    else if (j.dot4) *path = vktFilterPathDot8;
    else *path = vktFilterPathVectorFP32;
    if (products) *products = p;
    return vktNoError;
}

vktError vktSetAutotune(int enable)
{
    state().autotune = enable != 0;
    return vktNoError;
}

vktError vktSetStream(void* stream)
{
    state().stream = static_cast<hipStream_t>(stream);
    return vktNoError;
}

vktError vktGetStream(void** stream)
{
    if (!stream) return vktInvalidValue;
    *stream = state().stream;
    return vktNoError;
}

vktError vktSetPrecision(vktPrecision p)
{
    if (p < vktPrecisionAuto || p > vktPrecisionSplitBF16x6) return vktInvalidValue;
    state().precision = p;
    return vktNoError;
}

vktError vktGetPrecision(vktPrecision* p)
{
    if (!p) return vktInvalidValue;
    *p = state().precision;
    return vktNoError;
}

vktError vktSynchronize(void)
{
    hipError_t e = hipStreamSynchronize(state().stream);
    if (e == hipSuccess) e = hipGetLastError();
    return from_hip(e);
}

const char* vktGetErrorString(vktError e)
{
    switch (e) {
    case vktNoError: return "no error";
    case vktInvalidValue: return "invalid value";
    case vktOutOfMemory: return "out of device memory";
    case vktDeviceError: return "device error";
    case vktUnsupported: return "unsupported";
    }
    return "unknown error";
}

}  // extern "C"
