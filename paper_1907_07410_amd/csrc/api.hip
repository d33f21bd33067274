// The C ABI (include/bmf.h): argument checks, context state, and the
// sequencing of the device work.  Every entry point converts internal
// errors into bmf_status codes; no exception crosses the boundary.
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

using namespace bmf;

namespace {

thread_local std::string g_create_error;

template <class F>
bmf_status guarded(bmf_ctx *c, bool allow_poisoned, F &&f) {
    if (!c) return BMF_E_INVAL;
    if (c->poisoned && !allow_poisoned) {
        c->err = "context is poisoned by an earlier device error";
        return BMF_E_STATE;
    }
    try {
        BMF_HIP(hipSetDevice(c->M.device));
        f();
        return BMF_OK;
    } catch (const Error &e) {
        c->err = e.msg;
        if (e.code == BMF_E_DEVICE) c->poisoned = true;
        return e.code;
    } catch (const std::bad_alloc &) {
        c->err = "host allocation failed";
        return BMF_E_NOMEM;
    } catch (...) {
        c->err = "unexpected internal exception";
        c->poisoned = true;
        return BMF_E_DEVICE;
    }
}

HP hp_from(const float *h) { return HP{h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7]}; }
HP hp_uniform(float lr, float reg) { return HP{lr, reg, lr, reg, lr, reg, lr, reg}; }

void init_model_factors(Model &M) {
    launch_init_factors(M.P.as<float>(), M.m, M.k, M.seed, 1, M.stream);
    launch_init_factors(M.Q.as<float>(), M.n, M.k, M.seed, 2, M.stream);
    launch_fill(M.bu.as<float>(), M.m, 0.f, M.stream);
    launch_fill(M.bi.as<float>(), M.n, 0.f, M.stream);
    M.bf16_valid = false;
}

template <class T>
void upload(DevBuf &dst, const T *src, int64_t cnt, hipStream_t s) {
    dst.alloc((size_t)cnt * sizeof(T));
    if (cnt) BMF_HIP(hipMemcpyAsync(dst.p, src, (size_t)cnt * sizeof(T), hipMemcpyHostToDevice, s));
}

void check_finite_hp(const float *hp) {
    for (int q = 0; q < 8; ++q)
        if (!std::isfinite(hp[q])) BMF_FAIL(BMF_E_INVAL, "non-finite hyper-parameter");
}

// Partition (and, when an epoch will use it, plan) the device COO du/di/dr
// of nnz ratings for M's sizes, and make it the training set with mean mu.
// The buffers are taken over.
void set_training(Model &M, DevBuf &du, DevBuf &di, DevBuf &dr, int64_t nnz, double mu) {
    Partition P;
    build_partition(P, du.as<int32_t>(), di.as<int32_t>(), dr.as<float>(), nnz, M.m, M.n, M.b, M.stream);
    Plan plan;  // built now when an epoch will use it, else on first demand
    if (M.sgd_kernel == 2 || (M.sgd_kernel == 0 && plan_pays(P.nnz, M.b)))
        build_plan(plan, P, M.b, M.k, sgd_max_lds(M.device), M.stream);
    // a failure above leaves the model as it was; below, only a device error
    // (which poisons the context) can interrupt
    if (M.ooc.on) {  // kernels may still read its device buffers
        BMF_HIP(hipStreamSynchronize(M.stream));
        M.ooc.release();
    }
    M.cu.swap(du);
    M.ci.swap(di);
    M.cr.swap(dr);
    M.part.recs.swap(P.recs);
    M.part.perm.swap(P.perm);
    M.part.block_ptr.swap(P.block_ptr);
    M.part.h_block_ptr.swap(P.h_block_ptr);
    M.part.nnz = P.nnz;
    M.part.rb = P.rb;
    M.part.cb = P.cb;
    M.part.ibits = P.ibits;
    M.part.ubits = P.ubits;
    M.plan.swap(plan);
    M.mu = mu;
    M.loaded = true;
    M.bf16_valid = false;
}

// Copy a COO (host or device pointers) to new device buffers and check it
// against m x n; throws BMF_E_RANGE naming the first bad rating.
void stage_coo(Model &M, const int32_t *u, const int32_t *i, const float *r, int64_t nnz, bool dev, int64_t m,
               int64_t n, DevBuf &du, DevBuf &di, DevBuf &dr) {
    if (nnz < 0) BMF_FAIL(BMF_E_INVAL, "nnz < 0");
    if (nnz > 0 && (!u || !i || !r)) BMF_FAIL(BMF_E_INVAL, "null rating array");
    if (nnz >= (int64_t)INT32_MAX) BMF_FAIL(BMF_E_INVAL, "nnz must be below 2^31");
    du.alloc((size_t)nnz * 4);
    di.alloc((size_t)nnz * 4);
    dr.alloc((size_t)nnz * 4);
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (nnz) {
        BMF_HIP(hipMemcpyAsync(du.p, u, nnz * 4, kind, M.stream));
        BMF_HIP(hipMemcpyAsync(di.p, i, nnz * 4, kind, M.stream));
        BMF_HIP(hipMemcpyAsync(dr.p, r, nnz * 4, kind, M.stream));
    }
    const int64_t bad = validate_coo(du.as<int32_t>(), di.as<int32_t>(), dr.as<float>(), nnz, m, n, M.red,
                                     M.stream);
    if (bad >= 0) {
        std::string what = "rating " + std::to_string(bad) + " is out of range or not finite";
        if (!dev) what += " (u=" + std::to_string(u[bad]) + ", i=" + std::to_string(i[bad]) + ")";
        BMF_FAIL(BMF_E_RANGE, what);
    }
}

double training_mean(Model &M, const DevBuf &dr, int64_t nnz) {
    if (M.mu_mode != 0 || nnz == 0) return 0.0;
    return sum_f32_as_f64(dr.as<float>(), nnz, M.red, M.stream) / (double)nnz;
}

void load_common(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t nnz, bool dev) {
    Model &M = c->M;
    if (M.out_of_core) {
        if (dev) BMF_FAIL(BMF_E_INVAL, "out-of-core loads take host arrays");
        ooc_load(M, u, i, r, nnz);
        return;
    }
    DevBuf du, di, dr;
    stage_coo(M, u, i, r, nnz, dev, M.m, M.n, du, di, dr);
    set_training(M, du, di, dr, nnz, training_mean(M, dr, nnz));
}

// rows [r0, r1) of a k-wide factor table get their seeded initial values
void grow_table(DevBuf &A, int64_t r0, int64_t r1, int k, uint64_t seed, int tag, hipStream_t s) {
    DevBuf B;
    B.alloc((size_t)r1 * k * 4);
    if (r0) BMF_HIP(hipMemcpyAsync(B.p, A.p, (size_t)r0 * k * 4, hipMemcpyDeviceToDevice, s));
    launch_init_factors_rows(B.as<float>(), r0, r1, k, seed, tag, s);
    A.swap(B);
    BMF_HIP(hipStreamSynchronize(s));
}

void grow_bias(DevBuf &A, int64_t r0, int64_t r1, hipStream_t s) {
    DevBuf B;
    B.alloc((size_t)r1 * 4);
    if (r0) BMF_HIP(hipMemcpyAsync(B.p, A.p, (size_t)r0 * 4, hipMemcpyDeviceToDevice, s));
    launch_fill(B.as<float>() + r0, r1 - r0, 0.f, s);
    A.swap(B);
    BMF_HIP(hipStreamSynchronize(s));
}

// Sum of squared residuals over the training ratings (with the loss terms
// when loss_hp), resident or out of core.
double train_sq_sum(Model &M, const HP *loss_hp) {
    if (M.ooc.on) return ooc_sq_sum(M, loss_hp);
    return sq_residual_sum(M, M.cu.as<int32_t>(), M.ci.as<int32_t>(), M.cr.as<float>(), M.part.nnz, loss_hp, M.red);
}

void run_epoch(bmf_ctx *c, const HP &hp) {
    Model &M = c->M;
    if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
    std::vector<int32_t> order(M.b);
    schedule(M.b, M.order_seed, M.epoch, M.order_mode, order.data());
    sgd_epoch(M, order.data(), hp);
    M.epoch += 1;
    M.bf16_valid = false;
}

}  // namespace

extern "C" {

bmf_status bmf_create(int64_t m, int64_t n, int32_t k, int32_t b, bmf_ctx **out) {
    if (!out) return BMF_E_INVAL;
    *out = nullptr;
    if (m < 1 || n < 1 || k < 1 || k > 1024 || b < 1 || m >= INT32_MAX || n >= INT32_MAX) {
        g_create_error = "invalid sizes: need m, n in [1, 2^31), 1 <= k <= 1024, b >= 1";
        return BMF_E_INVAL;
    }
    if ((int64_t)b * b > (int64_t)1 << 26) {
        g_create_error = "block grid too large (b*b must be at most 2^26)";
        return BMF_E_INVAL;
    }
    bmf_ctx *c = new (std::nothrow) bmf_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return BMF_E_NOMEM;
    }
    try {
        Model &M = c->M;
        BMF_HIP(hipGetDevice(&M.device));
        BMF_HIP(hipStreamCreateWithFlags(&M.own_stream, hipStreamNonBlocking));
        M.stream = M.own_stream;
        M.m = m;
        M.n = n;
        M.k = k;
        M.b = b;
        M.P.alloc((size_t)m * k * 4);
        M.Q.alloc((size_t)n * k * 4);
        M.bu.alloc((size_t)m * 4);
        M.bi.alloc((size_t)n * 4);
        M.red.alloc(1 << 16);
        init_model_factors(M);
        BMF_HIP(hipStreamSynchronize(M.stream));
    } catch (const Error &e) {
        g_create_error = e.msg;
        bmf_destroy(c);
        return e.code == BMF_E_DEVICE ? BMF_E_DEVICE : e.code;
    } catch (...) {
        g_create_error = "unexpected internal exception";
        bmf_destroy(c);
        return BMF_E_DEVICE;
    }
    *out = c;
    return BMF_OK;
}

void bmf_destroy(bmf_ctx *c) {
    if (!c) return;
    Model &M = c->M;
    (void)hipSetDevice(M.device);
    if (M.stream) (void)hipStreamSynchronize(M.stream);
    for (auto &pr : M.pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (auto e : M.spare_events) (void)hipEventDestroy(e);
    if (M.own_stream) (void)hipStreamDestroy(M.own_stream);
    delete c;  // DevBuf destructors free device memory
}

const char *bmf_last_error(const bmf_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

bmf_status bmf_set_option(bmf_ctx *c, int32_t key, int64_t value) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        switch (key) {
        case BMF_OPT_SEED:
            M.seed = (uint64_t)value;
            init_model_factors(M);
            break;
        case BMF_OPT_ORDER_SEED: M.order_seed = (uint64_t)value; break;
        case BMF_OPT_STRATUM_ORDER:
            if (value != 0 && value != 1) BMF_FAIL(BMF_E_INVAL, "stratum order must be 0 or 1");
            M.order_mode = (int)value;
            break;
        case BMF_OPT_MU_MODE:
            if (value != 0 && value != 1) BMF_FAIL(BMF_E_INVAL, "mu mode must be 0 or 1");
            M.mu_mode = (int)value;
            break;
        case BMF_OPT_STREAM:
            BMF_HIP(hipStreamSynchronize(M.stream));
            M.stream = value ? reinterpret_cast<hipStream_t>(value) : M.own_stream;
            break;
        case BMF_OPT_SGD_KERNEL:
            if (value < 0 || value > 2) BMF_FAIL(BMF_E_INVAL, "SGD kernel must be 0, 1 or 2");
            M.sgd_kernel = (int)value;
            break;
        case BMF_OPT_WAVES_PER_BLOCK:
            if (value != 4 && value != 8) BMF_FAIL(BMF_E_INVAL, "waves per block must be 4 or 8");
            M.waves = (int)value;
            break;
        case BMF_OPT_OUT_OF_CORE:
            if (value != 0 && value != 1) BMF_FAIL(BMF_E_INVAL, "out-of-core must be 0 or 1");
            M.out_of_core = value == 1;
            break;
        case BMF_OPT_EPOCH:
            if (value < 0 || value >= (int64_t)INT32_MAX) BMF_FAIL(BMF_E_INVAL, "epoch must be in [0, 2^31 - 1)");
            M.epoch = (int)value;
            break;
        case BMF_OPT_EPOCH_GRAPH:
            if (value != 0 && value != 1) BMF_FAIL(BMF_E_INVAL, "epoch graph must be 0 or 1");
            BMF_HIP(hipStreamSynchronize(M.stream));
            M.egraph.reset();
            M.egraph.on = value == 1;
            break;
        default: BMF_FAIL(BMF_E_INVAL, "unknown option " + std::to_string(key));
        }
    });
}

bmf_status bmf_synchronize(bmf_ctx *c) {
    return guarded(c, false, [&] { BMF_HIP(hipStreamSynchronize(c->M.stream)); });
}

bmf_status bmf_load_ratings(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t nnz) {
    return guarded(c, false, [&] { load_common(c, u, i, r, nnz, false); });
}

bmf_status bmf_load_ratings_dev(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t nnz) {
    return guarded(c, false, [&] { load_common(c, u, i, r, nnz, true); });
}

bmf_status bmf_epoch(bmf_ctx *c, float lr, float reg) {
    return guarded(c, false, [&] {
        const float hp[8] = {lr, reg, lr, reg, lr, reg, lr, reg};
        check_finite_hp(hp);
        run_epoch(c, hp_uniform(lr, reg));
    });
}

bmf_status bmf_epoch_hp(bmf_ctx *c, const float hp[8]) {
    return guarded(c, false, [&] {
        if (!hp) BMF_FAIL(BMF_E_INVAL, "null hyper-parameters");
        check_finite_hp(hp);
        run_epoch(c, hp_from(hp));
    });
}

bmf_status bmf_fit(bmf_ctx *c, const float hp[8], int32_t max_epochs, double delta, int32_t *epochs_out,
                   double *rmse_out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!hp || max_epochs < 0 || !std::isfinite(delta)) BMF_FAIL(BMF_E_INVAL, "bad fit arguments");
        check_finite_hp(hp);
        if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
        const HP h = hp_from(hp);
        auto train_rmse = [&] {
            const int64_t nnz = M.part.nnz;
            if (nnz == 0) return 0.0;
            const double s = train_sq_sum(M, nullptr);
            return std::sqrt(s / (double)nnz);
        };
        double prev = train_rmse();
        int32_t done = 0;
        while (done < max_epochs) {
            run_epoch(c, h);
            ++done;
            const double cur = train_rmse();
            const bool improved = prev - cur >= delta;  // false also once the RMSE is not a number
            prev = cur;
            if (!improved) break;
        }
        if (epochs_out) *epochs_out = done;
        if (rmse_out) *rmse_out = prev;
    });
}

bmf_status bmf_add_ratings(bmf_ctx *c, int64_t m_new, int64_t n_new, const int32_t *u, const int32_t *i,
                           const float *r, int64_t nnz, const float hp[8], int32_t epochs_new) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (m_new < M.m || n_new < M.n || m_new >= INT32_MAX || n_new >= INT32_MAX)
            BMF_FAIL(BMF_E_INVAL, "the model can only grow, to sizes below 2^31");
        if (!hp || epochs_new < 0) BMF_FAIL(BMF_E_INVAL, "hp must be non-null and epochs_new >= 0");
        check_finite_hp(hp);
        if (M.ooc.on) BMF_FAIL(BMF_E_STATE, "incremental data needs resident ratings (load without out-of-core)");
        const int64_t old = M.loaded ? M.part.nnz : 0;
        if (nnz < 0 || old + nnz >= (int64_t)INT32_MAX) BMF_FAIL(BMF_E_INVAL, "nnz < 0 or the union reaches 2^31");
        DevBuf du, di, dr;
        stage_coo(M, u, i, r, nnz, false, m_new, n_new, du, di, dr);
        // union of the loaded ratings and the new ones, in that order
        const int64_t tot = old + nnz;
        DevBuf au, ai, ar;
        au.alloc((size_t)tot * 4);
        ai.alloc((size_t)tot * 4);
        ar.alloc((size_t)tot * 4);
        const DevBuf *src[2][3] = {{&M.cu, &M.ci, &M.cr}, {&du, &di, &dr}};
        DevBuf *dst[3] = {&au, &ai, &ar};
        for (int q = 0; q < 3; ++q) {
            char *d = static_cast<char *>(dst[q]->p);
            if (old) BMF_HIP(hipMemcpyAsync(d, src[0][q]->p, old * 4, hipMemcpyDeviceToDevice, M.stream));
            if (nnz) BMF_HIP(hipMemcpyAsync(d + old * 4, src[1][q]->p, nnz * 4, hipMemcpyDeviceToDevice, M.stream));
        }
        const double mu = training_mean(M, ar, tot);
        // grow the factor tables: kept rows, then seeded new rows and zero biases
        grow_table(M.P, M.m, m_new, M.k, M.seed, 1, M.stream);
        grow_table(M.Q, M.n, n_new, M.k, M.seed, 2, M.stream);
        grow_bias(M.bu, M.m, m_new, M.stream);
        grow_bias(M.bi, M.n, n_new, M.stream);
        M.m = m_new;
        M.n = n_new;
        M.Pb.free_();
        M.Qb.free_();
        M.bf16_valid = false;
        // the new ratings alone, on the grown grid, from the current factors
        if (epochs_new > 0 && nnz > 0) {
            set_training(M, du, di, dr, nnz, mu);
            for (int e = 0; e < epochs_new; ++e) run_epoch(c, hp_from(hp));
        }
        // then every rating is the training set
        set_training(M, au, ai, ar, tot, mu);
    });
}

bmf_status bmf_plan_info(bmf_ctx *c, int32_t *kernel, int64_t *steps, int32_t *slots, int64_t *block_steps) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
        int v = M.sgd_kernel;
        if (M.ooc.on && v == 0) v = M.ooc.variant;
        if (v == 0) v = M.plan.ok && plan_pays(M.part.nnz, M.b) ? 2 : 1;
        if (v == 2 && !M.ooc.on) ensure_plan(M);
        const bool planned = v == 2 && M.plan.ok;
        if (kernel) *kernel = v == 2 ? (planned ? 2 : 0) : (plan_kp(M.k) ? 1 : 3);
        if (steps) *steps = planned ? M.plan.total_steps : 0;
        if (slots) *slots = planned ? M.plan.S : 0;
        if (block_steps) {
            const int64_t nb = (int64_t)M.b * M.b;
            for (int64_t x = 0; x < nb; ++x)
                block_steps[x] = planned ? M.plan.h_blk_step[x + 1] - M.plan.h_blk_step[x] : 0;
        }
    });
}

bmf_status bmf_epoch_count(const bmf_ctx *c, int32_t *out) {
    if (!c || !out) return BMF_E_INVAL;
    *out = c->M.epoch;
    return BMF_OK;
}

bmf_status bmf_get_schedule(const bmf_ctx *c, int32_t epoch, int32_t *order) {
    if (!c || !order || epoch < 0) return BMF_E_INVAL;
    schedule(c->M.b, c->M.order_seed, epoch, c->M.order_mode, order);
    return BMF_OK;
}

bmf_status bmf_stratum_order(int32_t b, uint64_t seed, int32_t epoch, int32_t mode, int32_t *order) {
    if (b < 1 || !order || epoch < 0 || (mode != 0 && mode != 1)) return BMF_E_INVAL;
    schedule(b, seed, epoch, mode, order);
    return BMF_OK;
}

bmf_status bmf_get_partition(bmf_ctx *c, int64_t *block_ptr, int32_t *perm) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
        if (block_ptr)
            std::memcpy(block_ptr, M.part.h_block_ptr.data(), M.part.h_block_ptr.size() * sizeof(int64_t));
        if (perm && M.part.nnz && M.ooc.on) {
            std::memcpy(perm, M.ooc.perm.data(), M.part.nnz * 4);
        } else if (perm && M.part.nnz) {
            BMF_HIP(hipMemcpyAsync(perm, M.part.perm.p, M.part.nnz * 4, hipMemcpyDeviceToHost, M.stream));
            BMF_HIP(hipStreamSynchronize(M.stream));
        }
    });
}

bmf_status bmf_get_factors(bmf_ctx *c, float *P, float *Q, float *bu, float *bi, double *mu) {
    return guarded(c, true, [&] {
        Model &M = c->M;
        BMF_HIP(hipStreamSynchronize(M.stream));
        if (P) BMF_HIP(hipMemcpy(P, M.P.p, (size_t)M.m * M.k * 4, hipMemcpyDeviceToHost));
        if (Q) BMF_HIP(hipMemcpy(Q, M.Q.p, (size_t)M.n * M.k * 4, hipMemcpyDeviceToHost));
        if (bu) BMF_HIP(hipMemcpy(bu, M.bu.p, (size_t)M.m * 4, hipMemcpyDeviceToHost));
        if (bi) BMF_HIP(hipMemcpy(bi, M.bi.p, (size_t)M.n * 4, hipMemcpyDeviceToHost));
        if (mu) *mu = M.mu;
    });
}

bmf_status bmf_set_factors(bmf_ctx *c, const float *P, const float *Q, const float *bu, const float *bi,
                           const double *mu) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (mu && !std::isfinite(*mu)) BMF_FAIL(BMF_E_INVAL, "mu must be finite");
        BMF_HIP(hipStreamSynchronize(M.stream));
        if (P) BMF_HIP(hipMemcpy(M.P.p, P, (size_t)M.m * M.k * 4, hipMemcpyHostToDevice));
        if (Q) BMF_HIP(hipMemcpy(M.Q.p, Q, (size_t)M.n * M.k * 4, hipMemcpyHostToDevice));
        if (bu) BMF_HIP(hipMemcpy(M.bu.p, bu, (size_t)M.m * 4, hipMemcpyHostToDevice));
        if (bi) BMF_HIP(hipMemcpy(M.bi.p, bi, (size_t)M.n * 4, hipMemcpyHostToDevice));
        if (mu) M.mu = *mu;
        M.bf16_valid = false;
    });
}

bmf_status bmf_factor_ptrs(bmf_ctx *c, float **P, float **Q, float **bu, float **bi) {
    return guarded(c, false, [&] {
        if (P) *P = c->M.P.as<float>();
        if (Q) *Q = c->M.Q.as<float>();
        if (bu) *bu = c->M.bu.as<float>();
        if (bi) *bi = c->M.bi.as<float>();
        c->M.bf16_valid = false;  // the caller may write through these
    });
}

bmf_status bmf_rmse(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t cnt, double *out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!out) BMF_FAIL(BMF_E_INVAL, "null output");
        double s = 0.0;
        int64_t total = 0;
        if (!u) {
            if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
            total = M.part.nnz;
            s = train_sq_sum(M, nullptr);
        } else {
            if (cnt < 0 || (cnt > 0 && (!i || !r))) BMF_FAIL(BMF_E_INVAL, "bad evaluation arrays");
            for (int64_t t = 0; t < cnt; ++t)
                if (u[t] < 0 || u[t] >= M.m || i[t] < 0 || i[t] >= M.n || !std::isfinite(r[t]))
                    BMF_FAIL(BMF_E_RANGE, "evaluation rating " + std::to_string(t) + " out of range");
            DevBuf du, di, dr;
            upload(du, u, cnt, M.stream);
            upload(di, i, cnt, M.stream);
            upload(dr, r, cnt, M.stream);
            total = cnt;
            s = sq_residual_sum(M, du.as<int32_t>(), di.as<int32_t>(), dr.as<float>(), cnt, nullptr, M.red);
        }
        *out = total > 0 ? std::sqrt(s / (double)total) : 0.0;
    });
}

bmf_status bmf_rmse_dev(bmf_ctx *c, const int32_t *u, const int32_t *i, const float *r, int64_t cnt, double *out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!out) BMF_FAIL(BMF_E_INVAL, "null output");
        if (cnt < 0 || (cnt > 0 && (!u || !i || !r))) BMF_FAIL(BMF_E_INVAL, "bad evaluation arrays");
        const int64_t bad = validate_coo(u, i, r, cnt, M.m, M.n, M.red, M.stream);
        if (bad >= 0) BMF_FAIL(BMF_E_RANGE, "evaluation rating " + std::to_string(bad) + " out of range");
        const double s = cnt > 0 ? sq_residual_sum(M, u, i, r, cnt, nullptr, M.red) : 0.0;
        *out = cnt > 0 ? std::sqrt(s / (double)cnt) : 0.0;
    });
}

bmf_status bmf_loss(bmf_ctx *c, const float hp[8], double *out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!out || !hp) BMF_FAIL(BMF_E_INVAL, "null argument");
        if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
        const HP h = hp_from(hp);
        *out = train_sq_sum(M, &h);
    });
}

bmf_status bmf_check_disjoint(bmf_ctx *c, const int32_t *pairing, int64_t *conflicts) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (!conflicts) BMF_FAIL(BMF_E_INVAL, "null output");
        if (!M.loaded) BMF_FAIL(BMF_E_STATE, "no ratings loaded");
        if (M.ooc.on) BMF_FAIL(BMF_E_STATE, "the race check needs resident ratings");
        *conflicts = disjoint_check(M, sgd_variant(M), pairing);
    });
}

static void check_topk_args(const Model &M, int64_t nu, int32_t K, int32_t precision, int32_t Kc) {
    if (nu < 0) BMF_FAIL(BMF_E_INVAL, "nu < 0");
    if (K < 1 || K > 512) BMF_FAIL(BMF_E_INVAL, "K must be in [1, 512]");
    if (precision < 0 || precision > 2) BMF_FAIL(BMF_E_INVAL, "precision must be 0, 1 or 2");
    if (precision == 1 && Kc != 0 && (Kc < K || Kc > 1008)) BMF_FAIL(BMF_E_INVAL, "Kc must be 0 or in [K, 1008]");
    if (M.k > 256) BMF_FAIL(BMF_E_INVAL, "top-K scoring supports k <= 256");
}

static bmf_status topk_host(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t precision, int32_t Kc,
                            int32_t *items_out, float *scores_out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        check_topk_args(M, nu, K, precision, Kc);
        if (nu > 0 && (!users || !items_out || !scores_out)) BMF_FAIL(BMF_E_INVAL, "null array");
        for (int64_t q = 0; q < nu; ++q)
            if (users[q] < 0 || users[q] >= M.m) BMF_FAIL(BMF_E_RANGE, "user id " + std::to_string(users[q]) + " out of range");
        if (nu == 0) return;
        DevBuf du, di, ds;
        upload(du, users, nu, M.stream);
        di.alloc((size_t)nu * K * 4);
        ds.alloc((size_t)nu * K * 4);
        topk_run(M, du.as<int32_t>(), nu, K, precision, Kc, di.as<int32_t>(), ds.as<float>());
        BMF_HIP(hipMemcpyAsync(items_out, di.p, (size_t)nu * K * 4, hipMemcpyDeviceToHost, M.stream));
        BMF_HIP(hipMemcpyAsync(scores_out, ds.p, (size_t)nu * K * 4, hipMemcpyDeviceToHost, M.stream));
        BMF_HIP(hipStreamSynchronize(M.stream));
    });
}

bmf_status bmf_topk(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t *items_out, float *scores_out) {
    return topk_host(c, users, nu, K, 0, 0, items_out, scores_out);
}

bmf_status bmf_topk_bf16(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t Kc, int32_t *items_out,
                         float *scores_out) {
    return topk_host(c, users, nu, K, 1, Kc, items_out, scores_out);
}

bmf_status bmf_topk_dev(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t precision, int32_t Kc,
                        int32_t *items_out, float *scores_out) {
    return guarded(c, false, [&] {
        check_topk_args(c->M, nu, K, precision, Kc);
        if (nu > 0 && (!users || !items_out || !scores_out)) BMF_FAIL(BMF_E_INVAL, "null array");
        topk_run(c->M, users, nu, K, precision, Kc, items_out, scores_out);
    });
}

bmf_status bmf_topk_dev_noalloc(bmf_ctx *c, const int32_t *users, int64_t nu, int32_t K, int32_t precision,
                                int32_t Kc, int32_t *items_out, float *scores_out) {
    return guarded(c, false, [&] {
        check_topk_args(c->M, nu, K, precision, Kc);
        if (nu > 0 && (!users || !items_out || !scores_out)) BMF_FAIL(BMF_E_INVAL, "null array");
        topk_run_fixed(c->M, users, nu, K, precision, Kc, items_out, scores_out);
    });
}

bmf_status bmf_foldin(bmf_ctx *c, const int32_t *items, const float *r, int32_t nr, int32_t passes, float lr,
                      float reg, float *p_out, float *bu_out) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        if (nr < 0 || passes < 0 || !p_out || !bu_out || (nr > 0 && (!items || !r)))
            BMF_FAIL(BMF_E_INVAL, "bad fold-in arguments");
        if (!std::isfinite(lr) || !std::isfinite(reg)) BMF_FAIL(BMF_E_INVAL, "non-finite hyper-parameter");
        for (int32_t t = 0; t < nr; ++t)
            if (items[t] < 0 || items[t] >= M.n || !std::isfinite(r[t]))
                BMF_FAIL(BMF_E_RANGE, "fold-in rating " + std::to_string(t) + " out of range");
        DevBuf di, dr, dp, db;
        upload(di, items, nr, M.stream);
        upload(dr, r, nr, M.stream);
        dp.alloc((size_t)M.k * 4);
        db.alloc(4);
        foldin_run(M, di.as<int32_t>(), dr.as<float>(), nr, passes, hp_uniform(lr, reg), dp.as<float>(),
                   db.as<float>());
        BMF_HIP(hipMemcpy(p_out, dp.p, (size_t)M.k * 4, hipMemcpyDeviceToHost));
        BMF_HIP(hipMemcpy(bu_out, db.p, 4, hipMemcpyDeviceToHost));
    });
}

bmf_status bmf_sgd_timing(bmf_ctx *c, double *ms, int64_t *launches, int32_t reset) {
    return guarded(c, false, [&] {
        Model &M = c->M;
        harvest_timing(M, true);
        if (ms) *ms = M.sgd_ms;
        if (launches) *launches = M.sgd_launches;
        if (reset) {
            M.sgd_ms = 0.0;
            M.sgd_launches = 0;
        }
    });
}

bmf_status bmf_debug_topk_plan(int64_t n, int32_t k, int64_t nu, int32_t K, int32_t precision, int32_t Kc,
                               int64_t *out) {
    if (!out || n < 1 || k < 1 || k > 256 || nu < 1 || K < 1 || K > 512 || precision < 0 || precision > 2 ||
        (precision == 1 && Kc != 0 && (Kc < K || Kc > 1008)))
        return BMF_E_INVAL;
    try {
        const bmf::TopkPlan T = bmf::topk_plan(n, k, nu, K, precision, Kc);
        out[0] = T.s;
        out[1] = T.r;
        out[2] = T.capg;
        out[3] = T.Ksel;
        out[4] = T.S;
        out[5] = T.per_split;
        out[6] = (int64_t)T.total;
        return BMF_OK;
    } catch (const bmf::Error &e) {
        return e.code;
    } catch (...) {
        return BMF_E_NOMEM;
    }
}

bmf_status bmf_debug_block_plan(int64_t n, const int32_t *u_local, const int32_t *i_local, const float *r,
                                int32_t cb, int32_t slots, int32_t chunk, int64_t max_steps, int64_t *n_steps,
                                uint32_t *out) {
    if (n < 0 || (n > 0 && (!u_local || !i_local || !r)) || !n_steps || cb < 1 || cb >= (1 << 16) || slots < 1 ||
        slots > bmf::PLAN_MAX_SLOTS || chunk < 1)
        return BMF_E_INVAL;
    int ibits = 0;
    while ((1 << ibits) < cb) ++ibits;
    try {
        std::vector<uint32_t> ui(n);
        for (int64_t x = 0; x < n; ++x) {
            if (u_local[x] < 0 || (ibits > 0 && (uint64_t)u_local[x] >= (1ull << (32 - ibits))) || i_local[x] < 0 ||
                i_local[x] >= cb)
                return BMF_E_RANGE;
            if (x > 0 && (u_local[x] < u_local[x - 1] || (u_local[x] == u_local[x - 1] && i_local[x] < i_local[x - 1])))
                return BMF_E_INVAL;
            ui[x] = ((uint32_t)u_local[x] << ibits) | (uint32_t)i_local[x];
        }
        std::vector<bmf::PlanEntry> ent;
        const int64_t st = bmf::plan_block(ui.data(), n, ibits, cb, slots, chunk, ent);
        *n_steps = st;
        if (out) {
            if (max_steps < st) return BMF_E_RANGE;
            for (size_t q = 0; q < ent.size(); ++q) {
                uint32_t *o = out + 4 * q;
                const int64_t x = ent[q].x;
                if (x < 0) {
                    o[0] = (uint32_t)cb | ((uint32_t)slots << 16);
                    o[1] = 0u;
                    o[2] = 0u;
                    o[3] = 0xffffffffu;
                    continue;
                }
                const bool first = x == 0 || u_local[x - 1] != u_local[x];
                const bool last = x + 1 == n || u_local[x + 1] != u_local[x];
                o[0] = (uint32_t)i_local[x] | ((uint32_t)ent[q].slot << 16) | (first ? 1u << 30 : 0u) |
                       (last ? 1u << 31 : 0u);
                std::memcpy(&o[1], &r[x], 4);
                o[2] = (uint32_t)u_local[x];
                o[3] = (uint32_t)x;
            }
        }
    } catch (const bmf::Error &e) {
        g_create_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        return BMF_E_NOMEM;
    }
    return BMF_OK;
}

bmf_status bmf_debug_chain_floor(int32_t k, int32_t steps, double *ns_per_step) {
    if (k < 1 || k > 128 || steps < bmf::PLAN_CH || !ns_per_step) return BMF_E_INVAL;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float *d = nullptr;
    bmf_status st = BMF_OK;
    try {
        const int chunks = steps / bmf::PLAN_CH;
        BMF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        BMF_HIP(hipEventCreate(&e0));
        BMF_HIP(hipEventCreate(&e1));
        BMF_HIP(hipMalloc(&d, 8 * (128 + 4) * sizeof(float)));
        bmf::chain_floor(k, chunks, d, s);  // warm-up
        BMF_HIP(hipEventRecord(e0, s));
        bmf::chain_floor(k, chunks, d, s);
        BMF_HIP(hipEventRecord(e1, s));
        BMF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        BMF_HIP(hipEventElapsedTime(&ms, e0, e1));
        *ns_per_step = (double)ms * 1e6 / ((double)chunks * bmf::PLAN_CH);
    } catch (const Error &e) {
        g_create_error = e.msg;
        st = e.code;
    }
    if (d) (void)hipFree(d);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return st;
}

bmf_status bmf_chain_depth(int64_t n, const int32_t *u, const int32_t *i, int64_t *depth) {
    if (n < 0 || !depth || (n > 0 && (!u || !i))) return BMF_E_INVAL;
    for (int64_t x = 0; x < n; ++x)
        if (u[x] < 0 || i[x] < 0) return BMF_E_RANGE;
    try {
        *depth = bmf::chain_depth(u, i, n);
    } catch (const std::bad_alloc &) {
        return BMF_E_NOMEM;
    }
    return BMF_OK;
}

bmf_status bmf_debug_wave_sum(const float *in64, float *out256) {
    if (!in64 || !out256) return BMF_E_INVAL;
    try {
        DevBuf di, dout;
        di.alloc(64 * 4);
        dout.alloc(256 * 4);
        BMF_HIP(hipMemcpy(di.p, in64, 64 * 4, hipMemcpyHostToDevice));
        debug_wave_sum(di.as<float>(), dout.as<float>(), nullptr);
        BMF_HIP(hipMemcpy(out256, dout.p, 256 * 4, hipMemcpyDeviceToHost));
    } catch (const Error &e) {
        g_create_error = e.msg;
        return e.code;
    }
    return BMF_OK;
}

}  // extern "C"
