// tables.hip -- beam-splitter transition tables (Appendix), FP64.
//
// One thread per table entry.  Layout per gate: sectors N = 0..n_tab, each an
// (N+1) x (N+1) block stored x1-major: entry (x1, y1) of sector N sits at
// sector_offset(N) + x1 * (N+1) + y1 and holds <y1, N-y1| BS |x1, N-x1>.
#include "lofp_device.h"

namespace lofp {

// Entry idx of gate g's table (theta, phi of that gate).
__device__ double2 table_entry(int n_tab, int idx, double theta, double phi)
{
    if (idx >= sector_offset(n_tab + 1)) return make_double2(0.0, 0.0);   // the zero slot
    int N = 0;
    while (N < n_tab && sector_offset(N + 1) <= idx) ++N;
    const int rem = idx - sector_offset(N);
    const int x1 = rem / (N + 1), y1 = rem - x1 * (N + 1);
    const int x2 = N - x1, y2 = N - y1;
    double s, c;
    sincos(theta, &s, &c);
    // sum over t of (-1)^{y1-t} c^{x2-y1+2t} s^{x1+y1-2t} / (t!(y1-t)!(x1-t)!(x2-y1+t)!)
    const int tlo = (y1 - x2) > 0 ? (y1 - x2) : 0;
    const int thi = x1 < y1 ? x1 : y1;
    double sum = 0.0;
    for (int t = tlo; t <= thi; ++t) {
        double term = ipow(c, x2 - y1 + 2 * t) * ipow(s, x1 + y1 - 2 * t) /
                      (fact(t) * fact(y1 - t) * fact(x1 - t) * fact(x2 - y1 + t));
        sum += ((y1 - t) & 1) ? -term : term;
    }
    const double mag = sqrt(fact(x1) * fact(x2) * fact(y1) * fact(y2)) * sum;
    double sp, cp;
    sincos(phi * (double)(x1 - y1), &sp, &cp);
    return make_double2(mag * cp, mag * sp);
}

__global__ void k_build_tables(int G, int n_tab, int stride, const double *__restrict__ theta,
                               const double *__restrict__ phi, double2 *__restrict__ table)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)G * stride) return;
    const int g = (int)(k / stride);
    const int idx = (int)(k - (int64_t)g * stride);
    table[k] = table_entry(n_tab, idx, theta[g], phi[g]);
}

// Tables of many circuits: blockIdx.y picks the circuit.
__global__ void k_build_tables_multi(const TableJob *__restrict__ jobs)
{
    const TableJob j = jobs[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)j.G * j.stride) return;
    const int g = (int)(k / j.stride);
    const int idx = (int)(k - (int64_t)g * j.stride);
    j.table[k] = table_entry(j.n_tab, idx, j.theta[g], j.phi[g]);
}

hipError_t launch_build_tables(int G, int n_tab, const double *theta, const double *phi,
                               double2 *table, hipStream_t stream)
{
    const int stride = sector_offset(n_tab + 1) + 1;
    const int64_t total = (int64_t)G * stride;
    if (total == 0) return hipSuccess;
    const int block = 256;
    const int grid = (int)((total + block - 1) / block);
    hipLaunchKernelGGL(k_build_tables, dim3(grid), dim3(block), 0, stream, G, n_tab, stride, theta, phi,
                       table);
    return hipGetLastError();
}

hipError_t launch_build_tables_multi(int count, const TableJob *jobs, int64_t max_entries, hipStream_t stream)
{
    if (count == 0 || max_entries == 0) return hipSuccess;
    const int block = 256;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(k_build_tables_multi, dim3((unsigned)((max_entries + block - 1) / block), n), dim3(block),
                           0, stream, jobs + base);
    }
    return hipGetLastError();
}

}  // namespace lofp
