// The paper's frequency-domain Wiener step (Alg. 1, step d: wnrFn(adapOnly, original);
// Sec. III) on the device. With A = DFT2(a) of the AMF output and F = DFT2(f) of the clean
// original (H x W, the image's own size), the noise spectrum is N = A - F and every
// frequency is weighted by |F|^2 / (|F|^2 + |N|^2) (0 where both vanish); the output is
// real(IDFT2(gain A)) / M.
//
// 2-D DFT: one complex transform carries both real images (z = a + i f; A and F are the
// even and odd parts of Z(k) against conj(Z(-k))). Rows are transformed in LDS with
// Stockham autosort passes (radix 4, 2, 3, 5; twiddles from a table built in double
// precision), columns by transposing (32 x 32 LDS tiles) and transforming rows again. The
// inverse uses conj(DFT(conj(x))) and writes real(x) / (H W M) straight to the output.
#include "tile_io.h"

namespace hd {
namespace {

constexpr int FNT = 256;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // a * (-i)

// In-place forward DFT of R = 2, 3, 4, 5 points (kernel exp(-2 pi i r k / R)).
template <int R>
__device__ __forceinline__ void small_dft(float2 (&v)[5]) {
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else if constexpr (R == 3) {
        const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
        const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        const float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
        const float2 t = cscale(mul_mi(d), h);
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, t);
        v[2] = csub(m, t);
    } else {  // R == 5
        const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;  // cos(2pi/5), cos(4pi/5)
        const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;   // sin(2pi/5), sin(4pi/5)
        const float2 a = v[0];
        const float2 s14 = cadd(v[1], v[4]), d14 = csub(v[1], v[4]);
        const float2 s23 = cadd(v[2], v[3]), d23 = csub(v[2], v[3]);
        const float2 r1 = make_float2(a.x + c1 * s14.x + c2 * s23.x, a.y + c1 * s14.y + c2 * s23.y);
        const float2 r2 = make_float2(a.x + c2 * s14.x + c1 * s23.x, a.y + c2 * s14.y + c1 * s23.y);
        const float2 i1 = mul_mi(make_float2(s1 * d14.x + s2 * d23.x, s1 * d14.y + s2 * d23.y));
        const float2 i2 = mul_mi(make_float2(s2 * d14.x - s1 * d23.x, s2 * d14.y - s1 * d23.y));
        v[0] = cadd(a, cadd(s14, s23));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
}

// One Stockham pass of radix R over a length-n row: x -> y, span ns before the pass.
template <int R>
__device__ __forceinline__ void stockham_pass(const float2 *x, float2 *y, int n, int ns, const float2 *tw) {
    const int m = n / R;
    const int stride = n / (ns * R);  // twiddle exp(-2 pi i r k / (ns R)) = tw[r k stride]
    for (int j = threadIdx.x; j < m; j += FNT) {
        const int k = j % ns;
        float2 v[5];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[j + r * m];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * stride]);
        small_dft<R>(v);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) y[base + r * ns] = v[r];
    }
}

// Radix sequence of one transform length (4s first, then a 2, 3s, 5s).
struct FftPlan {
    int n, nst;
    int radix[14];
};

// Mode of the row transform's input / output.
enum RowIO : int {
    IO_COMPLEX = 0,     // complex rows in, complex rows out
    IO_OUT_REAL = 1,    // complex rows in, real part * scale to a float image out
};

// One workgroup per row: load (conjugated for the inverse), the passes in LDS, store.
__global__ __launch_bounds__(FNT) void fft_rows_kernel(float2 *data, long long pitch, FftPlan p,
                                                      const float2 *__restrict__ tw, int inverse, int io,
                                                      float *out, long long out_pitch, float scale) {
    extern __shared__ float2 sm[];
    const int n = p.n;
    float2 *x = sm, *y = sm + n;
    float2 *row = data + (long long)blockIdx.x * pitch;
    const float cj = inverse ? -1.0f : 1.0f;
    for (int i = threadIdx.x; i < n; i += FNT) {
        const float2 v = row[i];
        x[i] = make_float2(v.x, cj * v.y);
    }
    __syncthreads();
    int ns = 1;
    for (int st = 0; st < p.nst; ++st) {
        const int R = p.radix[st];
        if (R == 4) stockham_pass<4>(x, y, n, ns, tw);
        else if (R == 2) stockham_pass<2>(x, y, n, ns, tw);
        else if (R == 3) stockham_pass<3>(x, y, n, ns, tw);
        else stockham_pass<5>(x, y, n, ns, tw);
        __syncthreads();
        float2 *t = x;
        x = y;
        y = t;
        ns *= R;
    }
    if (io == IO_OUT_REAL) {
        float *o = out + (long long)blockIdx.x * out_pitch;
        for (int i = threadIdx.x; i < n; i += FNT) o[i] = x[i].x * scale;  // real part of conj(.)
    } else {
        for (int i = threadIdx.x; i < n; i += FNT) row[i] = make_float2(x[i].x, cj * x[i].y);
    }
}

// z[y][x] = (a[y][x], f[y][x]) as one complex image.
template <typename T>
__global__ __launch_bounds__(FNT) void pack_kernel(const T *__restrict__ a, long long ap, const T *__restrict__ f,
                                                  long long fp, float2 *z, int h, int w) {
    const long long n = (long long)h * w;
    for (long long i = (long long)blockIdx.x * FNT + threadIdx.x; i < n; i += (long long)gridDim.x * FNT) {
        const int y = (int)(i / w), x = (int)(i - (long long)y * w);
        z[i] = make_float2((float)a[(long long)y * ap + x], (float)f[(long long)y * fp + x]);
    }
}

// dst (cols x rows) = transpose of src (rows x cols), 32 x 32 tiles through LDS.
__global__ __launch_bounds__(FNT) void transpose_kernel(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                       int rows, int cols) {
    __shared__ float2 t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = 0; k < 32; k += 8) {
        const int r = by + ty + k, c = bx + tx;
        if (r < rows && c < cols) t[ty + k][tx] = src[(long long)r * cols + c];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int r = bx + ty + k, c = by + tx;  // dst row = src column
        if (r < cols && c < rows) dst[(long long)r * rows + c] = t[tx][ty + k];
    }
}

// Frequency-domain Wiener gain. zt holds Z = DFT2(a + i f) transposed: zt[kx][ky],
// W rows of H. A(k) = (Z(k) + conj(Z(-k))) / 2, F(k) = (Z(k) - conj(Z(-k))) / (2 i),
// N = A - F; q[kx][ky] = A |F|^2 / (|F|^2 + |N|^2).
__global__ __launch_bounds__(FNT) void wiener_gain_kernel(const float2 *__restrict__ zt, float2 *__restrict__ q,
                                                         int h, int w) {
    const long long n = (long long)h * w;
    for (long long i = (long long)blockIdx.x * FNT + threadIdx.x; i < n; i += (long long)gridDim.x * FNT) {
        const int kx = (int)(i / h), ky = (int)(i - (long long)kx * h);
        const int mx = kx == 0 ? 0 : w - kx, my = ky == 0 ? 0 : h - ky;
        const float2 z = zt[i], zm = zt[(long long)mx * h + my];
        const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        // (Z - conj(Zm)) / (2 i) = ((z.y + zm.y) - i (z.x - zm.x)) / 2
        const float2 F = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
        const float2 N = csub(A, F);
        const float pf = F.x * F.x + F.y * F.y;
        const float den = pf + (N.x * N.x + N.y * N.y);
        const float g = den > 0.0f ? pf / den : 0.0f;
        q[i] = cscale(A, g);
    }
}

__global__ void twiddle_kernel(float2 *tw, int n) {
    const int t = blockIdx.x * FNT + threadIdx.x;
    if (t >= n) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    tw[t] = make_float2((float)c, (float)(-s));  // exp(-2 pi i t / n)
}

bool fft_plan(int n, FftPlan *p) {
    if (n < 1 || n > FFT_MAX_LEN) return false;
    p->n = n;
    p->nst = 0;
    int m = n;
    while (m % 4 == 0) { p->radix[p->nst++] = 4; m /= 4; }
    while (m % 2 == 0) { p->radix[p->nst++] = 2; m /= 2; }
    while (m % 3 == 0) { p->radix[p->nst++] = 3; m /= 3; }
    while (m % 5 == 0) { p->radix[p->nst++] = 5; m /= 5; }
    return m == 1 && p->nst <= 14;
}

}  // namespace

bool fft_size_ok(int n) {
    FftPlan p;
    return fft_plan(n, &p);
}

// scratch: z (h w float2), zt (h w float2), twiddles (w + h float2)
size_t wiener_fft_scratch_bytes(int h, int w) {
    const size_t img = ((size_t)h * w * sizeof(float2) + 255) & ~(size_t)255;
    const size_t tws = (((size_t)w + h) * sizeof(float2) + 255) & ~(size_t)255;
    return 2 * img + tws;
}

hipError_t launch_wiener_fft(const void *a, long long ap, const void *f, long long fp, float *out, long long op,
                             int h, int w, int eb, int max_value, void *scratch, hipStream_t s) {
    FftPlan pw, ph;
    if (!fft_plan(w, &pw) || !fft_plan(h, &ph)) return hipErrorInvalidValue;
    const size_t img = ((size_t)h * w * sizeof(float2) + 255) & ~(size_t)255;
    float2 *z = (float2 *)scratch;
    float2 *zt = (float2 *)((char *)scratch + img);
    float2 *tww = (float2 *)((char *)scratch + 2 * img);
    float2 *twh = tww + w;
    const long long npx = (long long)h * w;
    const int eblocks = (int)((npx + FNT - 1) / FNT < 16384 ? (npx + FNT - 1) / FNT : 16384);
    hipLaunchKernelGGL(twiddle_kernel, dim3((w + FNT - 1) / FNT), dim3(FNT), 0, s, tww, w);
    hipLaunchKernelGGL(twiddle_kernel, dim3((h + FNT - 1) / FNT), dim3(FNT), 0, s, twh, h);
    if (eb == 1)
        hipLaunchKernelGGL(pack_kernel<uint8_t>, dim3(eblocks), dim3(FNT), 0, s, (const uint8_t *)a, ap,
                           (const uint8_t *)f, fp, z, h, w);
    else
        hipLaunchKernelGGL(pack_kernel<uint16_t>, dim3(eblocks), dim3(FNT), 0, s, (const uint16_t *)a, ap,
                           (const uint16_t *)f, fp, z, h, w);
    const dim3 tb(FNT);
    // forward: rows (length w), transpose to w x h, rows (length h)
    hipLaunchKernelGGL(fft_rows_kernel, dim3(h), tb, 2 * w * sizeof(float2), s, z, (long long)w, pw,
                       (const float2 *)tww, 0, (int)IO_COMPLEX, (float *)nullptr, 0ll, 1.0f);
    hipLaunchKernelGGL(transpose_kernel, dim3((w + 31) / 32, (h + 31) / 32), tb, 0, s, (const float2 *)z, zt, h, w);
    hipLaunchKernelGGL(fft_rows_kernel, dim3(w), tb, 2 * h * sizeof(float2), s, zt, (long long)h, ph,
                       (const float2 *)twh, 0, (int)IO_COMPLEX, (float *)nullptr, 0ll, 1.0f);
    // gain: zt (w x h) -> z used as q (w x h)
    hipLaunchKernelGGL(wiener_gain_kernel, dim3(eblocks), tb, 0, s, (const float2 *)zt, z, h, w);
    // inverse: rows of q (length h), transpose to h x w, rows (length w) -> real output
    hipLaunchKernelGGL(fft_rows_kernel, dim3(w), tb, 2 * h * sizeof(float2), s, z, (long long)h, ph,
                       (const float2 *)twh, 1, (int)IO_COMPLEX, (float *)nullptr, 0ll, 1.0f);
    hipLaunchKernelGGL(transpose_kernel, dim3((h + 31) / 32, (w + 31) / 32), tb, 0, s, (const float2 *)z, zt, w, h);
    const float scale = (float)(1.0 / ((double)h * (double)w * (double)max_value));
    hipLaunchKernelGGL(fft_rows_kernel, dim3(h), tb, 2 * w * sizeof(float2), s, zt, (long long)w, pw,
                       (const float2 *)tww, 1, (int)IO_OUT_REAL, out, op, scale);
    return hipGetLastError();
}

}  // namespace hd
