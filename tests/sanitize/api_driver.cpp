// Runs the C-ABI's host layer (api.cpp, linked with the launcher stand-ins of
// api_stubs.cpp) through every entry point, under AddressSanitizer and UBSan:
// size queries, argument checks and full calls whose launches only check that the
// workspace ranges they get lie inside the caller's workspace.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "fastqsl.h"

namespace fq {
extern const char *g_ws_lo, *g_ws_hi;
extern long g_calls;
}

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            fails++;                                                     \
        }                                                                \
    } while (0)

static double g_dummy[64];
static const void *fake_dev = g_dummy;  // device pointers are only passed through

static fq_field field(int nx, int ny, int nz, int dtype)
{
    fq_field f;
    memset(&f, 0, sizeof f);
    f.n[0] = nx, f.n[1] = ny, f.n[2] = nz;
    for (int a = 0; a < 3; a++) f.spacing[a] = 1.0 / (nx - 1), f.b[a] = fake_dev;
    f.dtype = dtype;
    return f;
}

static fq_plane plane(int nu, int nv, double z)
{
    fq_plane p;
    memset(&p, 0, sizeof p);
    p.origin[0] = 0.5 / nu, p.origin[1] = 0.5 / nv, p.origin[2] = z;
    p.u[0] = 1.0, p.v[1] = 1.0;
    p.nu = nu, p.nv = nv, p.du = 1.0 / nu, p.dv = 1.0 / nv;
    return p;
}

static std::vector<char> g_buf;
static void *workspace(size_t bytes)
{
    g_buf.assign(bytes + 512, 0);
    char *p = (char *)(((uintptr_t)g_buf.data() + 255) & ~(uintptr_t)255);
    fq::g_ws_lo = p;
    fq::g_ws_hi = p + bytes;
    return p;
}

static fq_map map_of(std::vector<double> &q, std::vector<double> &tw, std::vector<uint16_t> &st)
{
    fq_map m;
    memset(&m, 0, sizeof m);
    m.q = q.data(), m.tw = tw.data(), m.status = st.data();
    return m;
}

int main()
{
    for (int prec = 0; prec < 2; prec++)
        for (int dt = 0; dt < 2; dt++) {
            if (prec == FQ_PREC_F32X && dt == FQ_DT_F64 && false) continue;
            fq_params P;
            memset(&P, 0, sizeof P);
            P.precision = prec;
            P.want_tw = 1;
            // q2d, one job and a batch of three uneven jobs (one on an interior plane)
            fq_field f[3] = {field(33, 30, 17, dt), field(9, 9, 9, dt), field(64, 64, 40, dt)};
            fq_plane pl[3] = {plane(37, 29, 0.0), plane(3, 2, 0.0), plane(64, 64, 0.0)};
            std::vector<double> q(64 * 64), tw(64 * 64);
            std::vector<uint16_t> st(64 * 64);
            fq_map m[3] = {map_of(q, tw, st), map_of(q, tw, st), map_of(q, tw, st)};
            for (int nj = 1; nj <= 3; nj++) {
                size_t need = fastqsl_q2d_workspace_size(f, pl, nj, &P);
                CHECK(need > 0);
                void *ws = workspace(need);
                CHECK(fastqsl_q2d(f, pl, nj, &P, m, ws, need, nullptr) == FQ_OK);
                CHECK(fastqsl_q2d(f, pl, nj, &P, m, ws, need - 1, nullptr) == FQ_ENOMEM);
            }
            // Method II maps, and the fixed-step schemes
            fq_params P2 = P;
            P2.method = FQ_METHOD_II;
            for (int nj = 1; nj <= 3; nj++) {
                size_t need = fastqsl_q2d_workspace_size(f, pl, nj, &P2);
                CHECK(need > 0);
                CHECK(fastqsl_q2d(f, pl, nj, &P2, m, workspace(need), need, nullptr) == FQ_OK);
            }
            P2.scheme = FQ_SCHEME_RK4;
            CHECK(fastqsl_q2d_workspace_size(f, pl, 1, &P2) == 0);
            P2.method = FQ_METHOD_I;
            P2.scheme = FQ_SCHEME_RK4_38;
            {
                size_t need = fastqsl_q2d_workspace_size(f, pl, 2, &P2);
                CHECK(need > 0);
                CHECK(fastqsl_q2d(f, pl, 2, &P2, m, workspace(need), need, nullptr) == FQ_OK);
            }
            P2.scheme = 7;
            CHECK(fastqsl_q2d_workspace_size(f, pl, 1, &P2) == 0);
            // an interior plane (rotated S0) alone, and in a batch (unsupported)
            fq_plane mid = plane(20, 20, 0.37);
            size_t need = fastqsl_q2d_workspace_size(f, &mid, 1, &P);
            CHECK(need > 0);
            CHECK(fastqsl_q2d(f, &mid, 1, &P, m, workspace(need), need, nullptr) == FQ_OK);
            // interior planes in a batch: two rotated-S0 jobs beside a face plane
            fq_plane three[3] = {mid, pl[1], plane(11, 9, 0.21)};
            need = fastqsl_q2d_workspace_size(f, three, 3, &P);
            CHECK(need > 0);
            CHECK(fastqsl_q2d(f, three, 3, &P, m, workspace(need), need, nullptr) == FQ_OK);
            // q3d (Method I with rotated S0, and Method II)
            fq_voxels vx;
            memset(&vx, 0, sizeof vx);
            vx.n[0] = 11, vx.n[1] = 7, vx.n[2] = 5;
            for (int a = 0; a < 3; a++) vx.origin[a] = 0.05, vx.spacing[a] = 0.07;
            need = fastqsl_q3d_workspace_size(&f[0], &vx, &P);
            CHECK(need > 0);
            std::vector<double> q3(11 * 7 * 5), t3(11 * 7 * 5);
            std::vector<uint16_t> s3(11 * 7 * 5);
            fq_map m3 = map_of(q3, t3, s3);
            CHECK(fastqsl_q3d(&f[0], &vx, &P, &m3, workspace(need), need, nullptr) == FQ_OK);
            {
                fq_params P3 = P;
                P3.method = FQ_METHOD_II;
                size_t n3 = fastqsl_q3d_workspace_size(&f[0], &vx, &P3);
                CHECK(n3 > 0);
                CHECK(fastqsl_q3d(&f[0], &vx, &P3, &m3, workspace(n3), n3, nullptr) == FQ_OK);
            }
            // stretched grids: one stretched axis, and all three, in q2d (alone and in a
            // batch with a uniform job) and q3d; Method II there is unsupported
            {
                fq_field fs[2] = {field(33, 30, 17, dt), field(9, 9, 9, dt)};
                fs[0].coord[2] = (const double *)fake_dev;
                for (int all = 0; all < 2; all++) {
                    if (all) fs[0].coord[0] = fs[0].coord[1] = (const double *)fake_dev;
                    for (int nj = 1; nj <= 2; nj++) {
                        size_t ns_ = fastqsl_q2d_workspace_size(fs, pl, nj, &P);
                        CHECK(ns_ > 0);
                        CHECK(fastqsl_q2d(fs, pl, nj, &P, m, workspace(ns_), ns_, nullptr) == FQ_OK);
                    }
                    size_t n3 = fastqsl_q3d_workspace_size(&fs[0], &vx, &P);
                    CHECK(n3 > 0);
                    CHECK(fastqsl_q3d(&fs[0], &vx, &P, &m3, workspace(n3), n3, nullptr) == FQ_OK);
                    fq_params P4 = P;
                    P4.method = FQ_METHOD_II;
                    CHECK(fastqsl_q2d_workspace_size(fs, pl, 1, &P4) == 0);
                }
            }
            // cylinder maps (RKF45, Method I only; the cylinder inside the box in x, y)
            {
                fq_cylinder cy;
                memset(&cy, 0, sizeof cy);
                cy.centre[0] = 0.5, cy.centre[1] = 0.5, cy.radius = 0.3;
                cy.theta0 = 0.1, cy.dtheta = 0.05, cy.ntheta = 37, cy.z0 = 0.1, cy.dz = 0.05, cy.nz = 5;
                std::vector<double> qc(37 * 5), tc(37 * 5);
                std::vector<uint16_t> sc(37 * 5);
                fq_map mc = map_of(qc, tc, sc);
                size_t nc = fastqsl_qcyl_workspace_size(&f[0], &cy, &P);
                CHECK(nc > 0);
                CHECK(fastqsl_qcyl(&f[0], &cy, &P, &mc, workspace(nc), nc, nullptr) == FQ_OK);
                CHECK(fastqsl_qcyl(&f[0], &cy, &P, &mc, workspace(nc), nc - 1, nullptr) == FQ_ENOMEM);
                fq_params P5 = P;
                P5.method = FQ_METHOD_II;
                CHECK(fastqsl_qcyl_workspace_size(&f[0], &cy, &P5) == 0);
                P5 = P;
                P5.scheme = FQ_SCHEME_RK4;
                CHECK(fastqsl_qcyl_workspace_size(&f[0], &cy, &P5) == 0);
                cy.radius = 0.6;  // leaves the box in x
                CHECK(fastqsl_qcyl_workspace_size(&f[0], &cy, &P) == 0);
                CHECK(fastqsl_qcyl(&f[0], &cy, &P, &mc, workspace(nc), nc, nullptr) == FQ_EINVAL);
            }
            // trace lists, including an empty one
            fq_lines L;
            memset(&L, 0, sizeof L);
            need = fastqsl_trace_workspace_size(&f[0], 100, &P);
            CHECK(need > 0);
            CHECK(fastqsl_trace(&f[0], (const double *)fake_dev, 100, nullptr, &P, &L, workspace(need),
                                need, nullptr) == FQ_OK);
            CHECK(fastqsl_trace(&f[0], nullptr, 0, nullptr, &P, &L, nullptr, 0, nullptr) == FQ_OK);
            double zero_n[3] = {0, 0, 0};
            CHECK(fastqsl_trace(&f[0], (const double *)fake_dev, 1, zero_n, &P, &L, workspace(need),
                                need, nullptr) == FQ_EINVAL);
            // events recorded around the passes
            void *evs[4] = {(void *)1, (void *)2, (void *)3, (void *)4};
            P.events = evs;
            need = fastqsl_q2d_workspace_size(f, pl, 1, &P);
            CHECK(fastqsl_q2d(f, pl, 1, &P, m, workspace(need), need, nullptr) == FQ_OK);
            P.events = nullptr;
            // the adjoint: both precision forms, Method I, plane on a box face
            double *gb[3] = {g_dummy, g_dummy, g_dummy};
            need = fastqsl_backward_workspace_size(&f[0], &pl[0], &P, 32);
            {
                CHECK(need > 0);
                void *ws = workspace(need);
                CHECK(fastqsl_backward(&f[0], &pl[0], &P, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                       ws, need, nullptr) == FQ_OK);
                CHECK(fastqsl_q2d_record(&f[0], &pl[0], &P, 32, m, ws, need, nullptr) == FQ_OK);
                CHECK(fastqsl_backward_recorded(&f[0], &pl[0], &P, 32, g_dummy, nullptr, nullptr,
                                                nullptr, gb, ws, need, nullptr) == FQ_OK);
                // an interior plane: its rotated-S0 job's lines are differentiated too
                const size_t nmid = fastqsl_backward_workspace_size(&f[0], &mid, &P, 32);
                CHECK(nmid > 0);
                CHECK(fastqsl_backward(&f[0], &mid, &P, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                       workspace(nmid), nmid, nullptr) == FQ_OK);
                CHECK(fastqsl_q2d_record(&f[0], &mid, &P, 32, m, workspace(nmid), nmid, nullptr) == FQ_OK);
                CHECK(fastqsl_backward_recorded(&f[0], &mid, &P, 32, g_dummy, nullptr, nullptr, nullptr,
                                                gb, workspace(nmid), nmid, nullptr) == FQ_OK);
                fq_params P7 = P;
                P7.scheme = FQ_SCHEME_RK4;  // an interior plane's adjoint takes RKF45 only
                CHECK(fastqsl_backward_workspace_size(&f[0], &mid, &P7, 32) == 0);
                CHECK(fastqsl_backward_workspace_size(&f[0], &pl[0], &P, 0) == 0);
                // stretched grids have an adjoint too
                fq_field fst = f[0];
                fst.coord[1] = (const double *)fake_dev;
                const size_t nst = fastqsl_backward_workspace_size(&fst, &pl[0], &P, 32);
                CHECK(nst > 0);
                CHECK(fastqsl_backward(&fst, &pl[0], &P, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                       workspace(nst), nst, nullptr) == FQ_OK);
                P.tape_steps = 100000;
                size_t big = fastqsl_backward_workspace_size(&f[0], &pl[0], &P, 32);
                CHECK(big > need);
                P.tape_steps = -1;
                CHECK(fastqsl_backward_workspace_size(&f[0], &pl[0], &P, 32) == 0);
                P.tape_steps = 0;
                // the fixed-step schemes have an adjoint; Method II has none
                fq_params P6 = P;
                P6.scheme = FQ_SCHEME_RK4_38;
                const size_t n6 = fastqsl_backward_workspace_size(&f[0], &pl[0], &P6, 32);
                CHECK(n6 > 0);
                CHECK(fastqsl_backward(&f[0], &pl[0], &P6, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                       workspace(n6), n6, nullptr) == FQ_OK);
                P6 = P;
                P6.method = FQ_METHOD_II;
                CHECK(fastqsl_backward_workspace_size(&f[0], &pl[0], &P6, 32) == 0);
                // a voxel map's adjoint: the one-call and two-call forms; RKF45 only
                const size_t nvx = fastqsl_q3d_backward_workspace_size(&f[0], &vx, &P, 32);
                CHECK(nvx > 0);
                CHECK(fastqsl_q3d_backward(&f[0], &vx, &P, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                           workspace(nvx), nvx, nullptr) == FQ_OK);
                CHECK(fastqsl_q3d_record(&f[0], &vx, &P, 32, &m3, workspace(nvx), nvx, nullptr) == FQ_OK);
                CHECK(fastqsl_q3d_backward_recorded(&f[0], &vx, &P, 32, g_dummy, nullptr, nullptr,
                                                    nullptr, gb, workspace(nvx), nvx, nullptr) == FQ_OK);
                CHECK(fastqsl_q3d_backward(&f[0], &vx, &P, 32, g_dummy, g_dummy, nullptr, nullptr, gb,
                                           workspace(nvx), nvx - 1, nullptr) == FQ_ENOMEM);
                CHECK(fastqsl_q3d_record(&f[0], &vx, &P, 32, nullptr, workspace(nvx), nvx, nullptr) ==
                      FQ_EINVAL);
                CHECK(fastqsl_q3d_backward_workspace_size(&f[0], &vx, &P7, 32) == 0);
                CHECK(fastqsl_q3d_backward_workspace_size(&f[0], &vx, &P6, 32) == 0);
                CHECK(fastqsl_q3d_backward_workspace_size(&f[0], &vx, &P, 5000) == 0);
                CHECK(fastqsl_q3d_backward_workspace_size(&fst, &vx, &P, 32) > 0);
            }
            // argument checks
            {
                fq_params Pi = P;
                Pi.in_flight = 7;  // any nonzero value: the FP64 pass's shared-GPU form
                const size_t ni = fastqsl_q2d_workspace_size(f, pl, 1, &Pi);
                CHECK(ni > 0);
                CHECK(fastqsl_q2d(f, pl, 1, &Pi, m, workspace(ni), ni, nullptr) == FQ_OK);
                Pi.reserved2 = 1;
                CHECK(fastqsl_q2d_workspace_size(f, pl, 1, &Pi) == 0);
            }
            fq_field bad = f[0];
            bad.n[1] = 1;
            CHECK(fastqsl_q2d_workspace_size(&bad, pl, 1, &P) == 0);
            bad = f[0];
            bad.spacing[2] = -1.0;
            CHECK(fastqsl_q3d_workspace_size(&bad, &vx, &P) == 0);
            fq_plane skew = pl[0];
            skew.v[0] = 0.5;
            CHECK(fastqsl_q2d_workspace_size(f, &skew, 1, &P) == 0);
            fq_params badp = P;
            badp.block = 96;
            CHECK(fastqsl_q2d_workspace_size(f, pl, 1, &badp) == 0);
            CHECK(fastqsl_q2d(f, pl, 1, &P, nullptr, nullptr, 0, nullptr) == FQ_EINVAL);
            CHECK(fastqsl_q2d(f, pl, 0, &P, m, nullptr, 0, nullptr) == FQ_EINVAL);
        }
    CHECK(strcmp(fastqsl_strerror(FQ_ENOMEM), "workspace too small") == 0);
    CHECK(fastqsl_version() != nullptr);
    printf("api host layer: %ld launches checked, %d failures\n", fq::g_calls, fails);
    return fails ? 1 : 0;
}
