// Host-side setup of the library (topology, Hodge, plain and learned SPAI
// construction, stability limit, conjugate gradients, leapfrog energy
// guard, point location, absorbing layers) driven on a mesh file, for runs
// under the address and undefined-behaviour sanitizers.  Exit status 0 and
// one summary line; any sanitizer report ends the run with an error.
//
// Mesh file (little endian): int32 n_nodes, n_tris, n_seg; double zr[n_nodes][2];
// int32 tri[n_tris][3]; int32 seg[n_seg][2]; uint8 tag[n_seg].
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1701_03784_amd/csrc/host_setup.h"

using namespace axp;

static bool read_all(FILE *f, void *p, size_t size, size_t n) { return std::fread(p, size, n, f) == n; }

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[3];
    if (!read_all(f, hdr, 4, 3)) return 2;
    std::vector<double> zr(2 * size_t(hdr[0]));
    std::vector<int32_t> tri(3 * size_t(hdr[1])), seg(2 * size_t(hdr[2]));
    std::vector<uint8_t> tag(static_cast<size_t>(hdr[2]));
    if (!read_all(f, zr.data(), 8, zr.size()) || !read_all(f, tri.data(), 4, tri.size()) ||
        !read_all(f, seg.data(), 4, seg.size()) || !read_all(f, tag.data(), 1, tag.size()))
        return 2;
    std::fclose(f);
    try {
        HostMesh m;
        build_topology(m, hdr[0], zr.data(), hdr[1], tri.data(), hdr[2], seg.data(), tag.data());
        assemble_hodge(m);
        // plain SPAI at two levels, then the learned construction from a
        // perturbed copy of the plain columns (stands in for a network)
        build_spai(m, 2, 0.0, 3);
        const double fro2 = m.spai_fro;
        build_spai(m, 3, 1e-3, 3);
        const double fro3 = m.spai_fro;
        ScaledHodge h;
        scaled_hodge(m, h);
        PairSet ps;
        spai_pair_features(m, h, 3, 3, ps);
        std::vector<float> pred(ps.j.size());
        std::mt19937 rng(7);
        std::normal_distribution<float> noise(0.0f, 0.01f);
        for (size_t q = 0; q < pred.size(); ++q) pred[q] = (ps.X[16 * q] > 0.5f ? 1.0f : 0.0f) + noise(rng);
        ps.X.clear();
        LearnedSpaiStats st;
        learned_spai(m, h, ps, pred.data(), 3, 1e-3, 3, 0.02, 3, st);
        const double dt = cfl_dt(m, 200);
        const double drift = leapfrog_energy_drift(m, 0.5 * dt, 32, 11);
        // conjugate gradients for D = M^-1 E of a smooth field
        std::vector<double> E(m.n1), D(m.n1, 0.0);
        for (int e = 0; e < m.n1; ++e) E[e] = m.efree[e] ? std::sin(0.37 * e) : 0.0;
        const int it = cg_solve_M(m, E.data(), D.data(), 1e-12, 2000);
        // point location over the bounding box (points outside return -1)
        build_locator(m);
        double zmin = 1e300, zmax = -1e300, rmax = 0.0;
        for (int i = 0; i < hdr[0]; ++i) {
            zmin = std::fmin(zmin, zr[2 * i]);
            zmax = std::fmax(zmax, zr[2 * i]);
            rmax = std::fmax(rmax, zr[2 * i + 1]);
        }
        int inside = 0;
        for (int q = 0; q < 4000; ++q) {
            double lam[3];
            const double z = zmin + (zmax - zmin) * (q % 61) / 60.0, rho = rmax * (q / 61) / 65.0;
            if (locate_point(m, z, rho, lam) >= 0) ++inside;
        }
        // absorbing layers over the last fifth in z, and their stretched Hodge
        LayerConfig lc;
        lc.sides = 2;
        lc.z_right = zmax - 0.2 * (zmax - zmin);
        lc.sigma_max = 1e3;
        HostLayers L;
        Csr K;
        build_layers(m, 0.5 * dt, lc, L, K);
        std::printf("faces %d edges %d | SPAI fro L2 %.3e L3 %.3e learned fallback %lld | dt_cfl %.3e drift %.1e | "
                    "cg %d | located %d | layer faces %zu\n",
                    m.n2, m.n1, fro2, fro3, (long long)st.n_fallback, dt, drift, it, inside, L.face.size());
        if (!(drift < 1e-6) || it < 0 || inside == 0) return 1;
    } catch (const SetupError &e) {
        std::printf("setup error %d: %s\n", e.code, e.msg.c_str());
        return 3;
    }
    return 0;
}
