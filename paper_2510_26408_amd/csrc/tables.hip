// tables.hip -- beam-splitter transition tables (Appendix), FP64.
//
// Layout per gate: sectors N = 0..n_tab, each an (N+1) x (N+1) block stored
// x1-major: entry (x1, y1) of sector N sits at sector_offset(N) + x1 * (N+1)
// + y1 and holds <y1, N-y1| BS |x1, N-x1>; one zero entry closes the gate.
//
// The Appendix gives each entry as an alternating sum over t, whose terms
// grow like binomial coefficients while the entry stays below one, so in
// FP64 the sum loses about log2(max term) bits (3e-13 absolute near N = 30,
// 8e-12 near N = 40).  The tables are built instead from the same splitter
// acting on creation operators (the construction the Appendix starts from):
// a photon added to the upper input mode maps to U_aa a+ + U_ba b+ on the
// outputs, so
//   <y1, y2| BS |x1 + 1, x2> = ( U_aa sqrt(y1) <y1 - 1, y2| BS |x1, x2>
//                              + U_ba sqrt(y2) <y1, y2 - 1| BS |x1, x2> ) / sqrt(x1 + 1)
// and likewise for a photon added to the lower input with U_ab, U_bb.  The
// photon is always added to the fuller input mode (x1 >= x2: upper), so the
// factors sqrt(y) / sqrt(x) stay near one and rounding errors grow slowly
// (2.5e-14 at N = 64, where adding every photon on the upper side, or the
// closed form, loses 1e-8 or more).  With c = cos theta, s = sin theta the
// single-photon matrix of Eq. (bs_matrix) is U_aa = U_bb = c,
// U_ba = s e^{i phi} (upper in, lower out), U_ab = -s e^{-i phi}.
#include "lofp_device.h"

namespace lofp {

// All sectors of one gate's table by one block, in order of N (each sector
// reads the previous one, written by the same block before a barrier).
// theta NaN marks an exact mode swap (cos theta = 0, sin theta = phi = +-1,
// no phase), which the host uses to bring distant modes together.
__device__ void build_gate_table(int n_tab, double theta, double phi, double2 *__restrict__ tab)
{
    double s, c, sp, cp;
    if (isnan(theta)) {
        s = phi; c = 0.0; sp = 0.0; cp = 1.0;
    } else {
        sincos(theta, &s, &c);
        sincos(phi, &sp, &cp);
    }
    const double2 u_aa = make_double2(c, 0.0), u_bb = u_aa;
    const double2 u_ba = make_double2(s * cp, s * sp);     // upper in, lower out
    const double2 u_ab = make_double2(-s * cp, s * sp);    // lower in, upper out: -s e^{-i phi}
    if (threadIdx.x == 0) {
        tab[0] = make_double2(1.0, 0.0);                    // sector 0: the vacuum
        tab[sector_offset(n_tab + 1)] = make_double2(0.0, 0.0);   // the zero slot
    }
    __syncthreads();
    for (int N = 1; N <= n_tab; ++N) {
        const double2 *prev = tab + sector_offset(N - 1);
        double2 *cur = tab + sector_offset(N);
        for (int k = threadIdx.x; k < (N + 1) * (N + 1); k += blockDim.x) {
            const int x1 = k / (N + 1), x2 = N - x1, y1 = k - x1 * (N + 1), y2 = N - y1;
            // add the last photon to the fuller input; px1 is the upper input
            // of the sector N - 1 entry it starts from
            const bool up = x1 > 0 && x1 >= x2;
            const int px1 = up ? x1 - 1 : x1;
            const double2 ua = up ? u_aa : u_ab, ub = up ? u_ba : u_bb;
            const double inv = 1.0 / sqrt((double)(up ? x1 : x2));
            double2 acc = make_double2(0.0, 0.0);
            if (y1 > 0) {   // the new photon leaves through the upper output
                const double2 t = cmul(ua, prev[px1 * N + (y1 - 1)]);
                const double r = sqrt((double)y1);
                acc = make_double2(t.x * r, t.y * r);
            }
            if (y2 > 0) {   // through the lower output
                const double2 t = cmul(ub, prev[px1 * N + y1]);
                const double r = sqrt((double)y2);
                acc.x = fma(t.x, r, acc.x);
                acc.y = fma(t.y, r, acc.y);
            }
            cur[k] = make_double2(acc.x * inv, acc.y * inv);
        }
        __syncthreads();
    }
}

// Tables of many circuits: blockIdx.y picks the circuit, blockIdx.x the gate.
__global__ __launch_bounds__(256) void k_build_tables_multi(const TableJob *__restrict__ jobs)
{
    const TableJob j = jobs[blockIdx.y];
    const int g = blockIdx.x;
    if (g >= j.G) return;
    build_gate_table(j.n_tab, j.theta[g], j.phi[g], j.table + (int64_t)g * j.stride);
}

hipError_t launch_build_tables_multi(int count, const TableJob *jobs, int max_gates, hipStream_t stream)
{
    if (count == 0 || max_gates == 0) return hipSuccess;
    for (int base = 0; base < count; base += 65535) {
        const int n = count - base < 65535 ? count - base : 65535;
        hipLaunchKernelGGL(k_build_tables_multi, dim3((unsigned)max_gates, n), dim3(256), 0, stream, jobs + base);
    }
    return hipGetLastError();
}

}  // namespace lofp
