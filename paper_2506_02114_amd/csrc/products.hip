// Products of a map (sec. 4.1, 5): light curves of a point source moving
// along a straight track, and the distribution of log10 magnification.  Both
// read the map once and are bound by memory traffic.
#include "dev.hpp"

namespace mlm {

namespace {

constexpr int HIST_BLK = 256;
constexpr int HIST_MAX_LDS_BINS = 8192;   // bins kept in LDS per workgroup (64 KiB of u64)

// mu at source point (y1, y2): bilinear interpolation between the centres of
// the four nearest pixels; within half a pixel of the map's edge the nearest
// row or column is repeated; NaN outside the map
__device__ inline double interp(const double *__restrict__ mu, const MapGeom &g, double y1, double y2)
{
    const double u = (y1 - g.ylo1) / g.pix1, v = (y2 - g.ylo2) / g.pix2;
    if (!(u >= 0.0 && v >= 0.0 && u <= (double)g.n1 && v <= (double)g.n2)) return nan("");
    const double s = fmin(fmax(u - 0.5, 0.0), (double)(g.n1 - 1));
    const double t = fmin(fmax(v - 0.5, 0.0), (double)(g.n2 - 1));
    const int64_t i0 = (int64_t)fmin(floor(s), (double)(g.n1 - 1)), j0 = (int64_t)fmin(floor(t), (double)(g.n2 - 1));
    const int64_t i1 = i0 + 1 < g.n1 ? i0 + 1 : i0, j1 = j0 + 1 < g.n2 ? j0 + 1 : j0;
    const double fs = s - (double)i0, ft = t - (double)j0;
    const double a = mu[j0 * g.n1 + i0], b = mu[j0 * g.n1 + i1];
    const double c = mu[j1 * g.n1 + i0], d = mu[j1 * g.n1 + i1];
    return (1.0 - ft) * ((1.0 - fs) * a + fs * b) + ft * ((1.0 - fs) * c + fs * d);
}

// point k of npts evenly spaced from (y1a, y2a) to (y1b, y2b), both ends included
__global__ void k_light_curve(const double *__restrict__ mu, MapGeom g, double y1a, double y2a, double y1b,
                              double y2b, int64_t npts, double *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    const double f = npts > 1 ? (double)k / (double)(npts - 1) : 0.0;
    out[k] = interp(mu, g, y1a + f * (y1b - y1a), y2a + f * (y2b - y2a));
}

// bin of log10(mu): 0 underflow (mu <= 0 or below lo), 1 .. nbins the bins
// [lo + (b - 1) w, lo + b w), nbins + 1 overflow (and NaN)
__device__ inline int hist_bin(double m, double lo, double inv_w, int nbins)
{
    if (!(m > 0.0)) return isnan(m) ? nbins + 1 : 0;
    const double x = (log10(m) - lo) * inv_w;
    if (x < 0.0) return 0;
    if (!(x < (double)nbins)) return nbins + 1;
    return 1 + (int)x;
}

// counts per bin; a workgroup privatises the bins in LDS and adds them to
// the device counts once
__global__ __launch_bounds__(HIST_BLK) void k_histogram(const double *__restrict__ mu, int64_t npix, double lo,
                                                        double inv_w, int nbins,
                                                        unsigned long long *__restrict__ counts)
{
    extern __shared__ unsigned long long h[];
    const int nb = nbins + 2;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npix; k += stride)
        atomicAdd(&h[hist_bin(mu[k], lo, inv_w, nbins)], 1ull);
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        if (h[b]) atomicAdd(&counts[b], h[b]);
}

// the same without LDS, for more bins than a workgroup's LDS holds
__global__ void k_histogram_global(const double *__restrict__ mu, int64_t npix, double lo, double inv_w, int nbins,
                                   unsigned long long *__restrict__ counts)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < npix) atomicAdd(&counts[hist_bin(mu[k], lo, inv_w, nbins)], 1ull);
}

__global__ void k_zero_counts(unsigned long long *c, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) c[k] = 0;
}

}  // namespace

void launch_light_curve(const double *mu, const MapGeom &g, double y1a, double y2a, double y1b, double y2b,
                        int64_t npts, double *out, hipStream_t st)
{
    if (npts > 0)
        hipLaunchKernelGGL(k_light_curve, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, mu, g, y1a, y2a, y1b,
                           y2b, npts, out);
}

void launch_histogram(const double *mu, int64_t npix, double lo, double hi, int nbins, unsigned long long *counts,
                      hipStream_t st)
{
    const int nb = nbins + 2;
    hipLaunchKernelGGL(k_zero_counts, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, counts, nb);
    if (npix <= 0) return;
    const double inv_w = (double)nbins / (hi - lo);
    if (nb <= HIST_MAX_LDS_BINS) {
        // enough workgroups to fill the chip a few times over, each walking a
        // grid-strided share of the pixels
        const int64_t want = (npix + HIST_BLK * 16 - 1) / (HIST_BLK * 16);
        const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(want, 1), 2048);
        hipLaunchKernelGGL(k_histogram, dim3(grid), dim3(HIST_BLK), (size_t)nb * sizeof(unsigned long long), st, mu,
                           npix, lo, inv_w, nbins, counts);
    } else {
        hipLaunchKernelGGL(k_histogram_global, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, mu, npix, lo,
                           inv_w, nbins, counts);
    }
}

}  // namespace mlm
