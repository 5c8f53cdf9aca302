// Tikhonov-regularised deconvolution of recorded responses by the source function, the
// step (3) of the paper's route to the auxiliary responses (App. A-2), and the plain causal
// convolution of many series with one kernel (the one-run monostatic Jacobian):
//   G = conj(F) P / (|F|^2 + delta max|F|^2),   g = first N samples of IFFT(G),
// on the recorded window of N samples zero-padded to L = the smallest power of two
// >= 2N.  The transforms are batched real FFTs (hipFFT, in place, one series per padded
// row of 2 (L/2 + 1) reals); padding, the spectral filter and the truncation are kernels
// of this file.  Series are processed in chunks that bound the scratch memory.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <map>
#include <memory>
#include <tuple>
#include <cmath>
#include <complex>
#include <vector>

#include "mgrt_internal.hpp"
#include "series_filter.hpp"

namespace mgrt {

namespace {

#define MGRT_FFT(call)                                                                   \
    do {                                                                                  \
        hipfftResult r_ = (call);                                                         \
        if (r_ != HIPFFT_SUCCESS)                                                         \
            throw ::mgrt::Error(MGRT_E_HIP, std::string("hipFFT error ") + std::to_string((int)r_) + \
                                                " in " #call);                            \
    } while (0)

struct FftPlan {
    hipfftHandle h = 0;
    bool live = false;
    FftPlan() = default;
    FftPlan(const FftPlan &) = delete;
    FftPlan &operator=(const FftPlan &) = delete;
    void reset() {
        if (live) (void)hipfftDestroy(h);
        live = false;
    }
    ~FftPlan() { reset(); }
};

// buf[s][t] = x[s][t] for t < N, 0 up to the padded row length LP
template <typename T>
__global__ void k_pad_in(const T *__restrict__ x, int64_t N, int64_t LP, int64_t ns, T *__restrict__ buf) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = idx / LP, t = idx - s * LP;
    if (s >= ns) return;
    buf[idx] = t < N ? x[s * N + t] : T(0);
}

// spectrum row s: X[s][f] *= H[f]  (complex, interleaved)
template <typename T>
__global__ void k_spec_filter(T *__restrict__ X, const T *__restrict__ H, int64_t NF, int64_t ns) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = idx / NF, f = idx - s * NF;
    if (s >= ns) return;
    T *z = X + 2 * (s * NF + f);
    const T hr = H[2 * f], hi = H[2 * f + 1];
    const T xr = z[0], xi = z[1];
    z[0] = xr * hr - xi * hi;
    z[1] = xr * hi + xi * hr;
}

// x[s][t] = buf[s][t] / L for t < N
template <typename T>
__global__ void k_pad_out(const T *__restrict__ buf, int64_t N, int64_t LP, int64_t ns, T scale,
                          T *__restrict__ x) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = idx / N, t = idx - s * N;
    if (s >= ns) return;
    x[idx] = buf[s * LP + t] * scale;
}

template <typename T>
void make_plans(FftPlan &fwd, FftPlan &inv, int L, int64_t batch, hipStream_t s) {
    const int NF = L / 2 + 1, LP = 2 * NF;
    int n[1] = {L}, nr[1] = {LP}, nc[1] = {NF};
    const bool dbl = sizeof(T) == 8;
    MGRT_FFT(hipfftPlanMany(&fwd.h, 1, n, nr, 1, LP, nc, 1, NF, dbl ? HIPFFT_D2Z : HIPFFT_R2C, (int)batch));
    fwd.live = true;
    MGRT_FFT(hipfftPlanMany(&inv.h, 1, n, nc, 1, NF, nr, 1, LP, dbl ? HIPFFT_Z2D : HIPFFT_C2R, (int)batch));
    inv.live = true;
    MGRT_FFT(hipfftSetStream(fwd.h, s));
    MGRT_FFT(hipfftSetStream(inv.h, s));
}

// Plans are kept in the context: creating one costs about 12 ms of host work (and the
// first transform of a length compiles its kernels), against a few ms for the transforms
// of a whole Jacobian batch.  Each pair holds its own work area until the context ends.
struct PlanPair {
    FftPlan fwd, inv;
};
struct FftCache {
    std::map<std::tuple<int64_t, int64_t, int>, std::unique_ptr<PlanPair>> plans;
};

template <typename T>
PlanPair &cached_plans(Ctx &c, int64_t L, int64_t batch) {
    if (!c.fft_plans)
        c.fft_plans = std::shared_ptr<void>(new FftCache, [](void *p) { delete static_cast<FftCache *>(p); });
    auto &cache = static_cast<FftCache *>(c.fft_plans.get())->plans;
    const auto key = std::make_tuple(L, batch, (int)sizeof(T));
    auto it = cache.find(key);
    if (it == cache.end()) {
        auto pp = std::make_unique<PlanPair>();
        make_plans<T>(pp->fwd, pp->inv, (int)L, batch, c.stream);
        it = cache.emplace(key, std::move(pp)).first;
    }
    return *it->second;
}

// The plans of the cache are shared by callers on different streams: each execution
// names its stream.
template <typename T>
void exec_fwd(FftPlan &p, T *buf, hipStream_t s) {
    MGRT_FFT(hipfftSetStream(p.h, s));
    if constexpr (sizeof(T) == 8)
        MGRT_FFT(hipfftExecD2Z(p.h, reinterpret_cast<hipfftDoubleReal *>(buf),
                               reinterpret_cast<hipfftDoubleComplex *>(buf)));
    else
        MGRT_FFT(hipfftExecR2C(p.h, reinterpret_cast<hipfftReal *>(buf), reinterpret_cast<hipfftComplex *>(buf)));
}

template <typename T>
void exec_inv(FftPlan &p, T *buf, hipStream_t s) {
    MGRT_FFT(hipfftSetStream(p.h, s));
    if constexpr (sizeof(T) == 8)
        MGRT_FFT(hipfftExecZ2D(p.h, reinterpret_cast<hipfftDoubleComplex *>(buf),
                               reinterpret_cast<hipfftDoubleReal *>(buf)));
    else
        MGRT_FFT(hipfftExecC2R(p.h, reinterpret_cast<hipfftComplex *>(buf), reinterpret_cast<hipfftReal *>(buf)));
}

template <typename T>
void deconvolve_t(Ctx &c, T *x, int64_t n_series, int64_t N, const std::vector<double> &f, double delta,
                  size_t scratch_cap) {
    hipStream_t s = c.stream;
    int64_t L = 1;
    while (L < 2 * N) L *= 2;
    MGRT_REQUIRE(L <= (int64_t)1 << 30, MGRT_E_ARG, "series too long for the deconvolution");
    const int64_t NF = L / 2 + 1, LP = 2 * NF;
    // spectrum of the source function (FP64, one transform on the device)
    std::vector<double> F(2 * NF);
    {
        std::vector<double> fp(LP, 0.0);
        for (int64_t t = 0; t < N; ++t) fp[t] = f[t];
        DevBuf bf = upload(fp, s);
        exec_fwd<double>(cached_plans<double>(c, L, 1).fwd, bf.as<double>(), s);
        MGRT_HIP(hipMemcpyAsync(F.data(), bf.p, F.size() * 8, hipMemcpyDeviceToHost, s));
        MGRT_HIP(hipStreamSynchronize(s));
    }
    double f2max = 0.0;
    for (int64_t k = 0; k < NF; ++k) f2max = std::max(f2max, F[2 * k] * F[2 * k] + F[2 * k + 1] * F[2 * k + 1]);
    MGRT_REQUIRE(f2max > 0, MGRT_E_ARG, "the source function is zero on the recorded window");
    std::vector<T> H(2 * NF);
    for (int64_t k = 0; k < NF; ++k) {
        const double fr = F[2 * k], fi = F[2 * k + 1];
        const double den = fr * fr + fi * fi + delta * f2max;
        MGRT_REQUIRE(den > 0, MGRT_E_NONFINITE,
                     "the source spectrum vanishes where no regularisation is given (delta = 0)");
        H[2 * k] = (T)(fr / den);
        H[2 * k + 1] = (T)(-fi / den);
    }
    DevBuf dH = upload(H, s);
    // chunks of series through the padded scratch
    const int64_t per = LP * (int64_t)sizeof(T);
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_series, (int64_t)(scratch_cap / per)));
    DevBuf buf((size_t)chunk * per);
    for (int64_t s0 = 0; s0 < n_series; s0 += chunk) {
        const int64_t ns = std::min(chunk, n_series - s0);
        PlanPair &pp = cached_plans<T>(c, L, ns);
        FftPlan &fwd = pp.fwd, &inv = pp.inv;
        T *xs = x + s0 * N;
        hipLaunchKernelGGL(k_pad_in<T>, dim3((ns * LP + 255) / 256), dim3(256), 0, s, xs, N, LP, ns, buf.as<T>());
        exec_fwd<T>(fwd, buf.as<T>(), s);
        hipLaunchKernelGGL(k_spec_filter<T>, dim3((ns * NF + 255) / 256), dim3(256), 0, s, buf.as<T>(),
                           dH.as<T>(), NF, ns);
        exec_inv<T>(inv, buf.as<T>(), s);
        hipLaunchKernelGGL(k_pad_out<T>, dim3((ns * N + 255) / 256), dim3(256), 0, s, buf.as<T>(), N, LP, ns,
                           (T)(1.0 / (double)L), xs);
        MGRT_HIP(hipGetLastError());
    }
    MGRT_HIP(hipStreamSynchronize(s));
}

// buf[s][t] = (double) x[s][t] for t < N, 0 up to the padded row length LP
template <typename T>
__global__ void k_pad_in_d(const T *__restrict__ x, int64_t N, int64_t LP, int64_t ns, double *__restrict__ buf) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = idx / LP, t = idx - s * LP;
    if (s >= ns) return;
    buf[idx] = t < N ? (double)x[s * N + t] : 0.0;
}

// x[s][t] = (T) (buf[s][t] * scale) for t < N
template <typename T>
__global__ void k_pad_out_d(const double *__restrict__ buf, int64_t N, int64_t LP, int64_t ns, double scale,
                            T *__restrict__ x) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = idx / N, t = idx - s * N;
    if (s >= ns) return;
    x[idx] = (T)(buf[s * LP + t] * scale);
}

}  // namespace

struct SeriesFilter::Impl {
    int prec = 64;
    int64_t n_series = 0, N = 0, L = 1, NF = 0, LP = 0, chunk = 1;
    DevBuf dH, buf;
    PlanPair *full = nullptr, *tail = nullptr;   // plans for full chunks and the last one
};

// x[s] <- the first N samples of the causal convolution x[s] * h: rows zero-padded to
// L >= N + Mh - 1, FP64 real transforms, the product with the kernel's spectrum, the
// inverse, the first N samples scaled by 1/L.  Mh is h's length once its tail below
// 2^-60 of its largest magnitude is dropped (what is dropped changes an output by at most
// N 2^-60 max|h| max|x|, below the rounding of the FP64 transforms themselves), so that a
// short kernel takes shorter transforms; with L >= N + Mh - 1 nothing wraps into the first
// N samples.  L is the smallest power of two, or three times one (even), that suffices.
SeriesFilter::SeriesFilter(Ctx &c, int prec, int64_t n_series, int64_t N, const std::vector<double> &h,
                           size_t scratch_cap)
    : im_(new Impl) {
    Impl &m = *im_;
    MGRT_REQUIRE(prec == 32 || prec == 64, MGRT_E_ARG, "precision must be 32 or 64");
    MGRT_REQUIRE(n_series >= 1 && N >= 1 && (int64_t)h.size() >= N, MGRT_E_ARG, "empty convolution");
    m.prec = prec;
    m.n_series = n_series;
    m.N = N;
    double hmax = 0.0;
    for (int64_t t = 0; t < N; ++t) hmax = std::max(hmax, std::fabs(h[t]));
    int64_t Mh = N;
    while (Mh > 1 && !(std::fabs(h[Mh - 1]) > std::ldexp(hmax, -60))) --Mh;
    const int64_t need = std::max<int64_t>(2, N + Mh - 1);
    int64_t p2 = 2;
    while (p2 < need) p2 *= 2;
    m.L = p2 >= 8 && p2 / 4 * 3 >= need ? p2 / 4 * 3 : p2;   // even either way
    MGRT_REQUIRE(m.L <= (int64_t)1 << 30, MGRT_E_ARG, "series too long for the convolution");
    m.NF = m.L / 2 + 1;
    m.LP = 2 * m.NF;
    hipStream_t s = c.stream;
    {
        std::vector<double> hp(m.LP, 0.0);
        for (int64_t t = 0; t < Mh; ++t) hp[t] = h[t];
        m.dH = upload(hp, s);
        exec_fwd<double>(cached_plans<double>(c, m.L, 1).fwd, m.dH.as<double>(), s);
    }
    const int64_t per = m.LP * (int64_t)sizeof(double);
    m.chunk = std::max<int64_t>(1, std::min<int64_t>(n_series, (int64_t)(scratch_cap / per)));
    m.buf.alloc((size_t)m.chunk * per);
    m.full = &cached_plans<double>(c, m.L, m.chunk);
    if (n_series % m.chunk) m.tail = &cached_plans<double>(c, m.L, n_series % m.chunk);
    MGRT_HIP(hipStreamSynchronize(s));
}

SeriesFilter::~SeriesFilter() = default;

namespace {

template <typename T>
void filter_chunks(SeriesFilter::Impl &m, T *x, hipStream_t s) {
    double *buf = m.buf.as<double>();
    for (int64_t s0 = 0; s0 < m.n_series; s0 += m.chunk) {
        const int64_t ns = std::min(m.chunk, m.n_series - s0);
        PlanPair &pp = ns == m.chunk ? *m.full : *m.tail;
        T *xs = x + s0 * m.N;
        hipLaunchKernelGGL(k_pad_in_d<T>, dim3((ns * m.LP + 255) / 256), dim3(256), 0, s, xs, m.N, m.LP, ns, buf);
        exec_fwd<double>(pp.fwd, buf, s);
        hipLaunchKernelGGL(k_spec_filter<double>, dim3((ns * m.NF + 255) / 256), dim3(256), 0, s, buf,
                           m.dH.as<double>(), m.NF, ns);
        exec_inv<double>(pp.inv, buf, s);
        hipLaunchKernelGGL(k_pad_out_d<T>, dim3((ns * m.N + 255) / 256), dim3(256), 0, s, buf, m.N, m.LP, ns,
                           1.0 / (double)m.L, xs);
        MGRT_HIP(hipGetLastError());
    }
}

}  // namespace

void SeriesFilter::enqueue(void *x, hipStream_t s) {
    if (im_->prec == 32) filter_chunks<float>(*im_, static_cast<float *>(x), s);
    else filter_chunks<double>(*im_, static_cast<double *>(x), s);
}

void convolve_series(Ctx &c, void *x, int prec, int64_t n_series, int64_t N, const std::vector<double> &h,
                     size_t scratch_cap) {
    SeriesFilter f(c, prec, n_series, N, h, scratch_cap);
    f.enqueue(x, c.stream);
    MGRT_HIP(hipStreamSynchronize(c.stream));
}

void deconvolve_series(Ctx &c, void *x, int prec, int64_t n_series, int64_t N, const std::vector<double> &f,
                       double delta, size_t scratch_cap) {
    if (prec == 32) deconvolve_t<float>(c, static_cast<float *>(x), n_series, N, f, delta, scratch_cap);
    else deconvolve_t<double>(c, static_cast<double *>(x), n_series, N, f, delta, scratch_cap);
}

}  // namespace mgrt
