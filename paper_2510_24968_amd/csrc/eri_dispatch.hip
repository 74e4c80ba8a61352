// Quartet-class dispatch table over the per-class kernel files.
#include "fsim_internal.h"

namespace fsim {

hipError_t launch_eri_ssss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ssss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_psss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_psss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_psps_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_psps_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ppss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ppss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ppps_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ppps_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_pppp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_pppp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsps_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsps_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dspp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dspp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsds_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dsds_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpps_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpps_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dppp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dppp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpds_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpds_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpdp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dpdp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddss_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddss_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddps_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddps_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddpp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddpp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddds_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_ddds_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dddp_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dddp_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dddd_f64(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);
hipError_t launch_eri_dddd_f32(bool store, int variant, int wpb,
                               const EriArgs &a, hipStream_t s);

hipError_t launch_eri(int bra_pc, int ket_pc, bool fp32, bool store, int variant, int wpb,
                      const EriArgs &a, hipStream_t s) {
    switch (bra_pc * 8 + ket_pc) {
        case 0: return fp32 ? launch_eri_ssss_f32(store, variant, wpb, a, s)
                         : launch_eri_ssss_f64(store, variant, wpb, a, s);
        case 8: return fp32 ? launch_eri_psss_f32(store, variant, wpb, a, s)
                         : launch_eri_psss_f64(store, variant, wpb, a, s);
        case 9: return fp32 ? launch_eri_psps_f32(store, variant, wpb, a, s)
                         : launch_eri_psps_f64(store, variant, wpb, a, s);
        case 16: return fp32 ? launch_eri_ppss_f32(store, variant, wpb, a, s)
                         : launch_eri_ppss_f64(store, variant, wpb, a, s);
        case 17: return fp32 ? launch_eri_ppps_f32(store, variant, wpb, a, s)
                         : launch_eri_ppps_f64(store, variant, wpb, a, s);
        case 18: return fp32 ? launch_eri_pppp_f32(store, variant, wpb, a, s)
                         : launch_eri_pppp_f64(store, variant, wpb, a, s);
        case 24: return fp32 ? launch_eri_dsss_f32(store, variant, wpb, a, s)
                         : launch_eri_dsss_f64(store, variant, wpb, a, s);
        case 25: return fp32 ? launch_eri_dsps_f32(store, variant, wpb, a, s)
                         : launch_eri_dsps_f64(store, variant, wpb, a, s);
        case 26: return fp32 ? launch_eri_dspp_f32(store, variant, wpb, a, s)
                         : launch_eri_dspp_f64(store, variant, wpb, a, s);
        case 27: return fp32 ? launch_eri_dsds_f32(store, variant, wpb, a, s)
                         : launch_eri_dsds_f64(store, variant, wpb, a, s);
        case 32: return fp32 ? launch_eri_dpss_f32(store, variant, wpb, a, s)
                         : launch_eri_dpss_f64(store, variant, wpb, a, s);
        case 33: return fp32 ? launch_eri_dpps_f32(store, variant, wpb, a, s)
                         : launch_eri_dpps_f64(store, variant, wpb, a, s);
        case 34: return fp32 ? launch_eri_dppp_f32(store, variant, wpb, a, s)
                         : launch_eri_dppp_f64(store, variant, wpb, a, s);
        case 35: return fp32 ? launch_eri_dpds_f32(store, variant, wpb, a, s)
                         : launch_eri_dpds_f64(store, variant, wpb, a, s);
        case 36: return fp32 ? launch_eri_dpdp_f32(store, variant, wpb, a, s)
                         : launch_eri_dpdp_f64(store, variant, wpb, a, s);
        case 40: return fp32 ? launch_eri_ddss_f32(store, variant, wpb, a, s)
                         : launch_eri_ddss_f64(store, variant, wpb, a, s);
        case 41: return fp32 ? launch_eri_ddps_f32(store, variant, wpb, a, s)
                         : launch_eri_ddps_f64(store, variant, wpb, a, s);
        case 42: return fp32 ? launch_eri_ddpp_f32(store, variant, wpb, a, s)
                         : launch_eri_ddpp_f64(store, variant, wpb, a, s);
        case 43: return fp32 ? launch_eri_ddds_f32(store, variant, wpb, a, s)
                         : launch_eri_ddds_f64(store, variant, wpb, a, s);
        case 44: return fp32 ? launch_eri_dddp_f32(store, variant, wpb, a, s)
                         : launch_eri_dddp_f64(store, variant, wpb, a, s);
        case 45: return fp32 ? launch_eri_dddd_f32(store, variant, wpb, a, s)
                         : launch_eri_dddd_f64(store, variant, wpb, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsim
