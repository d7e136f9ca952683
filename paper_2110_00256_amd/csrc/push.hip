// Particle push in prescribed analytic fields, for closing the loop of the
// QED sub-step without a field solver (the benchmark geometries of the
// paper's Sec. 5.1: a static magnetic field perpendicular to the electrons,
// and a circularly polarised plane wave counter-propagating with them).
//
// Leptons: relativistic Boris rotation (u = p/(m_e c) at half steps,
// positions at whole steps): u- = u + eps E, rotation by t = (q dt/(2 m
// gamma-)) B, u+ = rotated u- + eps E, eps = q dt/(2 m c); x += c u dt/gamma.
// Photons move on straight lines at c.  After the move the fields at the new
// position and time are written to the particle's E/B arrays, which is what
// the QED step then reads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "constants.hpp"
#include "internal.hpp"

namespace qedmi {
namespace {

struct PushArgs {
    SetDev set;
    void *x, *y, *z;
    qed_field f;
    double t_new;    // time of the positions after the push
    double dt;
    double qm;       // q / m_e (C/kg), sign included; 0 for photons
};

__device__ __forceinline__ void field_at(const qed_field& f, double x, double t, double e[3], double b[3]) {
    if (f.kind == QED_FIELD_UNIFORM) {
        for (int k = 0; k < 3; ++k) {
            e[k] = f.e0[k];
            b[k] = f.b0[k];
        }
        return;
    }
    // circular polarisation, propagating along direction * x
    const double kw = 2.0 * 3.141592653589793 / f.wavelength;
    const double ph = kw * (f.direction * x - kC * t) + f.phase;
    const double c = cos(ph), s = sin(ph);
    e[0] = 0.0;
    e[1] = f.amplitude * c;
    e[2] = f.amplitude * s;
    // B = (direction x_hat) x E / c
    b[0] = 0.0;
    b[1] = -f.direction * e[2] / kC;
    b[2] = f.direction * e[1] / kC;
}

template <typename T>
__global__ void __launch_bounds__(256) push_kernel(PushArgs a) {
    const SetDev& S = a.set;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < S.n; i += int64_t(gridDim.x) * blockDim.x) {
        double u[3] = {static_cast<const T*>(S.p[0])[i], static_cast<const T*>(S.p[1])[i],
                       static_cast<const T*>(S.p[2])[i]};
        double r[3] = {static_cast<const T*>(a.x)[i], static_cast<const T*>(a.y)[i], static_cast<const T*>(a.z)[i]};
        if (a.qm != 0.0) {
            double e[3], b[3];
            field_at(a.f, r[0], a.t_new - a.dt, e, b);
            const double eps = a.qm * a.dt / (2.0 * kC);
            double um[3];
            for (int k = 0; k < 3; ++k) um[k] = u[k] + eps * e[k];
            const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
            double tv[3];
            for (int k = 0; k < 3; ++k) tv[k] = a.qm * a.dt / (2.0 * gm) * b[k];
            const double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
            double sv[3];
            for (int k = 0; k < 3; ++k) sv[k] = 2.0 * tv[k] / (1.0 + t2);
            const double up[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]), um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                                  um[2] + (um[0] * tv[1] - um[1] * tv[0])};
            double uplus[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]), um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                               um[2] + (up[0] * sv[1] - up[1] * sv[0])};
            for (int k = 0; k < 3; ++k) u[k] = uplus[k] + eps * e[k];
            const double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int k = 0; k < 3; ++k) r[k] += kC * u[k] / g * a.dt;
        } else {
            const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (um > 0.0)
                for (int k = 0; k < 3; ++k) r[k] += kC * u[k] / um * a.dt;
        }
        double e[3], b[3];
        field_at(a.f, r[0], a.t_new, e, b);
        for (int k = 0; k < 3; ++k) {
            static_cast<T*>(S.p[k])[i] = static_cast<T>(u[k]);
            static_cast<T*>(S.p[3 + k])[i] = static_cast<T>(e[k]);
            static_cast<T*>(S.p[6 + k])[i] = static_cast<T>(b[k]);
        }
        static_cast<T*>(a.x)[i] = static_cast<T>(r[0]);
        static_cast<T*>(a.y)[i] = static_cast<T>(r[1]);
        static_cast<T*>(a.z)[i] = static_cast<T>(r[2]);
    }
}

}  // namespace
}  // namespace qedmi

using namespace qedmi;

extern "C" int32_t qed_push(qed_context* ctx, const qed_particles* p, void* x, void* y, void* z,
                            const qed_field* field, double t, double dt, void* stream) {
    if (!ctx || !p || !field) { set_error("context/particles/field is null"); return QED_ERR_INVALID; }
    if (p->n < 0 || (p->dtype != QED_FP64 && p->dtype != QED_FP32)) { set_error("bad particles"); return QED_ERR_INVALID; }
    if (field->kind != QED_FIELD_UNIFORM && field->kind != QED_FIELD_CP_WAVE) { set_error("unknown field kind"); return QED_ERR_INVALID; }
    if (field->kind == QED_FIELD_CP_WAVE && (!(field->wavelength > 0.0) || (field->direction != 1 && field->direction != -1))) {
        set_error("CP wave needs wavelength > 0 and direction +-1");
        return QED_ERR_INVALID;
    }
    if (!(dt >= 0.0)) { set_error("dt < 0"); return QED_ERR_INVALID; }
    if (p->species == QED_ION) { set_error("ions are not pushed here"); return QED_ERR_INVALID; }
    if (p->n == 0) return QED_OK;
    const void* req[9] = {p->ux, p->uy, p->uz, p->ex, p->ey, p->ez, p->bx, p->by, p->bz};
    for (const void* q : req)
        if (!q) { set_error("a particle array pointer is null"); return QED_ERR_INVALID; }
    if (!x || !y || !z) { set_error("position arrays are null"); return QED_ERR_INVALID; }
    PushArgs a{};
    void* arr[11] = {p->ux, p->uy, p->uz, p->ex, p->ey, p->ez, p->bx, p->by, p->bz, p->tau, p->w};
    for (int i = 0; i < 11; ++i) a.set.p[i] = arr[i];
    a.set.n = p->n;
    a.x = x;
    a.y = y;
    a.z = z;
    a.f = *field;
    a.t_new = t + dt;
    a.dt = dt;
    a.qm = p->species == QED_ELECTRON ? -kQe / kMe : p->species == QED_POSITRON ? kQe / kMe : 0.0;
    const int64_t blocks = std::min<int64_t>((p->n + 255) / 256, 65536);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->dtype == QED_FP64)
        hipLaunchKernelGGL(push_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(push_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("qed_push launch: ") + hipGetErrorString(e));
        return QED_ERR_HIP;
    }
    return QED_OK;
}
