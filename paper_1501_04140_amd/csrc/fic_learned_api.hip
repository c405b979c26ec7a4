// Host runtime and C ABI of the learned domain proposal (included by
// fic_lib.hip, whose helpers it uses). Training and inference run entirely in
// the kernels of fic_mlp_kernels.hip; the exhaustive fallback reuses the
// level matcher.

struct fic_mlp {
    int device = 0;
    float tau = 0.1f;
    int step = 0;
    float* w = nullptr;  // fp32 master parameters
    float* m = nullptr;  // Adam moments
    float* v = nullptr;
    float* g = nullptr;  // last gradient
    _Float16* w16 = nullptr;
    uint32_t* maxbits = nullptr;
    fic::Buf X, H1, H2, Y, G32, nrm, G16, Z, Pm, Pt, GDt, GRt, dG, dS, dY, D1, D2, T1, T2, part,
        sums, loss, keys, cand, fbq, tmpm, tkq, tkgm, tkth, tkcnt;
};

namespace fic {
namespace {

// Grow a buffer of the network (every queued kernel is finished first).
int mgrow(Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (b.cap >= bytes) return FIC_OK;
    if (b.p) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = ((bytes + bytes / 4) + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FIC_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    b.cap = want;
    return FIC_OK;
}

inline int rup(int64_t a, int64_t b) { return (int)((a + b - 1) / b * b); }

template <int EPI>
void gemm(const _Float16* A, int lda, const _Float16* B, int ldb, int M, int N, int K, int splits,
          float alpha, const float* bias, const _Float16* mask, int ldm, void* C, int ldc,
          hipStream_t st) {
    const int kchunk = rup(cdiv(K, splits), 32);
    const int nz = cdiv(K, kchunk);
    // x: column blocks fastest, so that the workgroups sharing a block of A rows
    // run together and its re-reads come from L2
    k_gemm_nt<EPI><<<dim3(cdiv(M, 64) * cdiv(N, 64), 1, nz), 256, 0, st>>>(
        A, lda, B, ldb, M, N, kchunk, K, alpha, bias, mask, ldm, C, ldc);
}

// split count that gives about `want` workgroups over an M x N output
int splits_for(int M, int N, int K, int want = 1024) {
    const int tiles = cdiv(M, 64) * cdiv(N, 64);
    return std::max(1, std::min(cdiv(want, tiles), cdiv(K, 512)));
}

int k_splits(int K, int splits) { return cdiv(K, rup(cdiv(K, splits), 32)); }

__global__ void k_sum_parts(const float* __restrict__ part, int splits, int count, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
    out[i] = s;
}

// rows = 8 * nblk rows of X -> H1, H2, Y -> embeddings G16 (and G32, nrm)
int mlp_forward(fic_mlp* M, int nblk, bool keep, hipStream_t st) {
    const int64_t rows = (int64_t)nblk * 8;
    if (rows > INT32_MAX / 2) return fail(FIC_EINVAL, "too many blocks (%d)", nblk);
    int rc;
    if ((rc = mgrow(M->G16, (int64_t)nblk * 64 * 2))) return rc;
    if (!keep) {
        // no backward pass follows: the hidden layers and Y never leave the chip
        // persistent: about one workgroup of 8 waves per CU
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, M->device));
        const int tiles = (int)cdiv(rows, kFuseRows);
        k_mlp_forward<<<std::max(1, std::min(tiles, cus)), kFuseWaves * 64, 0, st>>>(
            P<_Float16>(M->X), (int)rows, M->w16, M->w, P<_Float16>(M->G16));
        LAUNCH_CHECK();
        return FIC_OK;
    }
    if ((rc = mgrow(M->Y, rows * kMlpOut * 4))) return rc;
    if ((rc = mgrow(M->H1, rows * kMlpHid * 2)) || (rc = mgrow(M->H2, rows * kMlpHid * 2))) return rc;
    if (keep && ((rc = mgrow(M->G32, (int64_t)nblk * 64 * 4)) || (rc = mgrow(M->nrm, (int64_t)nblk * 4))))
        return rc;
    const _Float16* X = P<_Float16>(M->X);
    _Float16* H1 = P<_Float16>(M->H1);
    _Float16* H2 = P<_Float16>(M->H2);
    const int R = (int)rows;
    gemm<kEpiRelu16>(X, 64, M->w16 + kH16W1, 64, R, kMlpHid, 64, 1, 1.0f, M->w + kOffB1, nullptr, 0, H1,
                     kMlpHid, st);
    gemm<kEpiRelu16>(H1, kMlpHid, M->w16 + kH16W2, kMlpHid, R, kMlpHid, kMlpHid, 1, 1.0f, M->w + kOffB2,
                     nullptr, 0, H2, kMlpHid, st);
    gemm<kEpiF32>(H2, kMlpHid, M->w16 + kH16W3, kMlpHid, R, kMlpOut, kMlpHid, 1, 1.0f, M->w + kOffB3,
                  nullptr, 0, P<float>(M->Y), kMlpOut, st);
    k_iso_norm<<<cdiv((int64_t)nblk * 64, 256), 256, 0, st>>>(
        P<float>(M->Y), nblk, keep ? P<float>(M->G32) : nullptr, keep ? P<float>(M->nrm) : nullptr,
        P<_Float16>(M->G16));
    LAUNCH_CHECK();
    return FIC_OK;
}

int check_block_image(const uint8_t* img, int H, int W, int pitch, int L) {
    if (!img) return fail(FIC_EINVAL, "image pointer is NULL");
    if (H < 16 || W < 16 || H % 8 || W % 8)
        return fail(FIC_EINVAL, "image %dx%d: sides must be multiples of 8 and >= 16", H, W);
    if (H > FIC_MAX_SIDE || W > FIC_MAX_SIDE) return fail(FIC_EINVAL, "image side above %d", FIC_MAX_SIDE);
    if (pitch < W) return fail(FIC_EINVAL, "pitch %d < width %d", pitch, W);
    if (L < 1) return fail(FIC_EINVAL, "domain step L=%d < 1", L);
    return FIC_OK;
}

// Block rows of n ranges (list = corners or NULL for the grid) then all domains.
int block_rows(fic_mlp* M, const uint8_t* img, int H, int W, int pitch, int L,
               const int32_t* range_yx, int nr, int nd, hipStream_t st) {
    const int gx = (W - 16) / L + 1;
    int rc = mgrow(M->X, ((int64_t)nr + nd) * 8 * 64 * 2);
    if (rc) return rc;
    _Float16* X = P<_Float16>(M->X);
    if (nr)
        k_block_rows<<<cdiv((int64_t)nr * 64, 256), 256, 0, st>>>(img, pitch, H, W, 0, L, gx, nd,
                                                                 range_yx, nr, X);
    if (nd)
        k_block_rows<<<cdiv((int64_t)nd * 64, 256), 256, 0, st>>>(img, pitch, H, W, 1, L, gx, nd,
                                                                 nullptr, nd, X + (int64_t)nr * 512);
    LAUNCH_CHECK();
    return FIC_OK;
}

// Top-k of GR [nq x 64] against GD [nk x 64] -> idx, score [nq x k]: the
// common scale and the int8 codes, the group maxima, theta, the lists, their
// merge.
int topk_launch(fic_mlp* M, const _Float16* GR, int nq, const _Float16* GD, int nk, int k,
                int32_t* idx, float* score, hipStream_t st) {
    if (nq <= 0) return FIC_OK;
    const int xb = cdiv(nq, kTkQ);
    // about 1024 workgroups; chunks of at least one stage of keys
    int nc = std::max(1, std::min(16, cdiv(1024, xb)));
    nc = std::max(1, std::min(nc, nk / kTkCols));
    const int G = 16 * nc;
    int rc;
    if ((rc = mgrow(M->tkq, 256 + ((int64_t)nq + nk) * 64)) || (rc = mgrow(M->tkgm, (int64_t)nq * G * 4)) ||
        (rc = mgrow(M->tkth, (int64_t)nq * 4)) || (rc = mgrow(M->keys, (int64_t)nc * nq * kTkCap * 8)) ||
        (rc = mgrow(M->tkcnt, (int64_t)nc * nq * 4)))
        return rc;
    uint32_t* mbits = P<uint32_t>(M->tkq);
    int8_t* QR = P<int8_t>(M->tkq) + 256;
    int8_t* QD = QR + (int64_t)nq * 64;
    int32_t* gm = P<int32_t>(M->tkgm);
    int32_t* th = P<int32_t>(M->tkth);
    uint64_t* list = P<uint64_t>(M->keys);
    int32_t* cnt = P<int32_t>(M->tkcnt);
    const int64_t nr8 = (int64_t)nq * 8, nk8 = (int64_t)nk * 8;
    k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(mbits), 1, 0);
    k_tk_absmax<<<(int)std::min<int64_t>(1024, cdiv(nr8 + nk8, 256)), 256, 0, st>>>(GR, nr8 * 8, GD, nk8 * 8, mbits);
    k_tk_quant<<<cdiv(nr8, 256), 256, 0, st>>>(GR, nr8, mbits, QR);
    if (nk > 0) k_tk_quant<<<cdiv(nk8, 256), 256, 0, st>>>(GD, nk8, mbits, QD);
    k_tk_max<<<dim3(xb, nc), kTkWaves * 64, 0, st>>>(QR, nq, QD, nk, gm);
    k_tk_theta<<<cdiv((int64_t)nq * 64, 256), 256, 0, st>>>(gm, nq, G, th);
    k_tk_collect<<<dim3(xb, nc), kTkWaves * 64, 0, st>>>(QR, nq, QD, nk, th, list, cnt);
    k_tk_merge<<<cdiv((int64_t)nq * 64, 256), 256, 0, st>>>(list, cnt, nc, nq, k, idx, score);
    LAUNCH_CHECK();
    return FIC_OK;
}

// Gradient of the mean cross-entropy into M->g (and the mean loss into loss_out).
int loss_grad_impl(fic_mlp* M, const uint8_t* img, int H, int W, int pitch, int L,
                   const int32_t* range_yx, const int32_t* labels, int nr, float* loss_out,
                   hipStream_t st) {
    const int gx = (W - 16) / L + 1, gy = (H - 16) / L + 1;
    const int nd = gx * gy;
    const int nb = nr + nd;
    const int rows = nb * 8;
    const int nd_pad = rup(nd, 32), nr_pad = rup(nr, 32), rows_pad = rup(rows, 32);
    int rc;
    if ((rc = block_rows(M, img, H, W, pitch, L, range_yx, nr, nd, st))) return rc;
    if ((rc = mlp_forward(M, nb, true, st))) return rc;
    if ((rc = mgrow(M->Z, (int64_t)nr * nd_pad * 4)) || (rc = mgrow(M->Pm, (int64_t)nr * nd_pad * 2)) ||
        (rc = mgrow(M->Pt, (int64_t)nd_pad * nr_pad * 2)) || (rc = mgrow(M->GDt, (int64_t)64 * nd_pad * 2)) ||
        (rc = mgrow(M->GRt, (int64_t)64 * nr_pad * 2)) || (rc = mgrow(M->dG, (int64_t)nb * 64 * 4)) ||
        (rc = mgrow(M->dS, (int64_t)nb * 64 * 4)) || (rc = mgrow(M->dY, (int64_t)rows * 64 * 2)) ||
        (rc = mgrow(M->D1, (int64_t)rows * kMlpHid * 2)) || (rc = mgrow(M->D2, (int64_t)rows * kMlpHid * 2)) ||
        (rc = mgrow(M->T1, (int64_t)kMlpHid * rows_pad * 2)) ||
        (rc = mgrow(M->T2, (int64_t)kMlpHid * rows_pad * 2)) || (rc = mgrow(M->loss, (int64_t)nr * 4)) ||
        (rc = mgrow(M->sums, 1024 * 4)))
        return rc;
    const _Float16* G16 = P<_Float16>(M->G16);
    const _Float16* GR = G16;
    const _Float16* GD = G16 + (int64_t)nr * 64;
    float* Z = P<float>(M->Z);
    _Float16* Pm = P<_Float16>(M->Pm);
    const float itau = 1.0f / M->tau;
    // similarities, softmax cross-entropy
    gemm<kEpiF32>(GR, 64, GD, 64, nr, nd, 64, 1, itau, nullptr, nullptr, 0, Z, nd_pad, st);
    k_softmax_ce<<<nr, 256, 0, st>>>(Z, nd_pad, nd, labels, Pm, nd_pad, P<float>(M->loss));
    if (loss_out) k_mean<<<1, 256, 0, st>>>(P<float>(M->loss), nr, loss_out);
    // dG_R = P G_D / tau, dG_D = P^T G_R / tau (gradient of the summed loss)
    k_transpose16<<<dim3(cdiv(nd_pad, 64), 1), 256, 0, st>>>(GD, 64, nd, 64, P<_Float16>(M->GDt), nd_pad, nd_pad);
    k_transpose16<<<dim3(cdiv(nr_pad, 64), 1), 256, 0, st>>>(GR, 64, nr, 64, P<_Float16>(M->GRt), nr_pad, nr_pad);
    k_transpose16<<<dim3(cdiv(nr_pad, 64), cdiv(nd_pad, 64)), 256, 0, st>>>(Pm, nd_pad, nr, nd_pad,
                                                                             P<_Float16>(M->Pt), nr_pad, nr_pad);
    float* dG = P<float>(M->dG);
    {
        int s = splits_for(nr, 64, nd_pad);
        const int z = k_splits(nd_pad, s);
        if ((rc = mgrow(M->part, (int64_t)z * nr * 64 * 4))) return rc;
        gemm<kEpiPart32>(Pm, nd_pad, P<_Float16>(M->GDt), nd_pad, nr, 64, nd_pad, s, itau, nullptr, nullptr, 0,
                         P<float>(M->part), 64, st);
        k_sum_parts<<<cdiv(nr * 64, 256), 256, 0, st>>>(P<float>(M->part), z, nr * 64, dG);
    }
    {
        int s = splits_for(nd, 64, nr_pad);
        const int z = k_splits(nr_pad, s);
        if ((rc = mgrow(M->part, (int64_t)z * nd * 64 * 4))) return rc;
        gemm<kEpiPart32>(P<_Float16>(M->Pt), nr_pad, P<_Float16>(M->GRt), nr_pad, nd, 64, nr_pad, s, itau, nullptr,
                         nullptr, 0, P<float>(M->part), 64, st);
        k_sum_parts<<<cdiv(nd * 64, 256), 256, 0, st>>>(P<float>(M->part), z, nd * 64, dG + (int64_t)nr * 64);
    }
    // back through the normalisation and the isometry sum
    k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(M->maxbits), 1, 0);
    k_norm_bwd<<<cdiv((int64_t)nb * 64, 256), 256, 0, st>>>(dG, P<float>(M->G32), P<float>(M->nrm), nb,
                                                            P<float>(M->dS), M->maxbits);
    _Float16* dY = P<_Float16>(M->dY);
    k_expand_grad<<<cdiv((int64_t)rows * 64, 256), 256, 0, st>>>(P<float>(M->dS), nb, M->maxbits, dY);
    // back through the three layers
    const float scale = 1.0f / (float)nr;
    _Float16* T1 = P<_Float16>(M->T1);
    _Float16* T2 = P<_Float16>(M->T2);
    float* sums = P<float>(M->sums);
    auto weight_grad = [&](const _Float16* dOut, int nout, const _Float16* In, int nin, int off) -> int {
        k_transpose16<<<dim3(cdiv(rows_pad, 64), cdiv(nout, 64)), 256, 0, st>>>(dOut, nout, rows, nout, T1,
                                                                                 rows_pad, rows_pad);
        k_transpose16<<<dim3(cdiv(rows_pad, 64), cdiv(nin, 64)), 256, 0, st>>>(In, nin, rows, nin, T2,
                                                                                rows_pad, rows_pad);
        const int s = splits_for(nout, nin, rows_pad);
        const int z = k_splits(rows_pad, s);
        int rc2 = mgrow(M->part, (int64_t)z * nout * nin * 4);
        if (rc2) return rc2;
        gemm<kEpiPart32>(T1, rows_pad, T2, rows_pad, nout, nin, rows_pad, s, 1.0f, nullptr, nullptr, 0,
                         P<float>(M->part), nin, st);
        k_grad_reduce<<<cdiv(nout * nin, 256), 256, 0, st>>>(P<float>(M->part), z, nout * nin, scale,
                                                             M->maxbits, M->g + off);
        k_row_sums<<<nout, 256, 0, st>>>(T1, rows_pad, rows, sums);
        // bias follows its weight matrix in the parameter layout
        k_scale_into<<<cdiv(nout, 256), 256, 0, st>>>(sums, nout, scale, M->maxbits, M->g + off + nout * nin);
        return FIC_OK;
    };
    _Float16* H1 = P<_Float16>(M->H1);
    _Float16* H2 = P<_Float16>(M->H2);
    _Float16* D2 = P<_Float16>(M->D2);
    _Float16* D1 = P<_Float16>(M->D1);
    if ((rc = weight_grad(dY, kMlpOut, H2, kMlpHid, kOffW3))) return rc;
    gemm<kEpiMask16>(dY, kMlpOut, M->w16 + kH16W3t, kMlpOut, rows, kMlpHid, kMlpOut, 1, 1.0f, nullptr, H2,
                     kMlpHid, D2, kMlpHid, st);
    if ((rc = weight_grad(D2, kMlpHid, H1, kMlpHid, kOffW2))) return rc;
    gemm<kEpiMask16>(D2, kMlpHid, M->w16 + kH16W2t, kMlpHid, rows, kMlpHid, kMlpHid, 1, 1.0f, nullptr, H1,
                     kMlpHid, D1, kMlpHid, st);
    if ((rc = weight_grad(D1, kMlpHid, P<_Float16>(M->X), kMlpIn, kOffW1))) return rc;
    LAUNCH_CHECK();
    return FIC_OK;
}

int adam_impl(fic_mlp* M, const float* grad, float lr, float b1, float b2, float eps, hipStream_t st) {
    M->step += 1;
    const double bc1 = 1.0 - std::pow((double)b1, M->step);
    const double bc2 = 1.0 - std::pow((double)b2, M->step);
    k_adam<<<cdiv(kMlpParams, 256), 256, 0, st>>>(M->w, M->m, M->v, grad ? grad : M->g, lr, b1, b2, eps,
                                                   (float)bc1, (float)bc2, M->w16);
    LAUNCH_CHECK();
    return FIC_OK;
}

int check_adam(float lr, float b1, float b2, float eps) {
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(FIC_EINVAL, "lr must be finite and > 0");
    if (!(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f))
        return fail(FIC_EINVAL, "beta1, beta2 must be in [0, 1)");
    if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(FIC_EINVAL, "eps must be finite and > 0");
    return FIC_OK;
}

}  // namespace
}  // namespace fic

FIC_API int fic_mlp_create(const float* init, float tau, fic_mlp** out) {
    if (!out) return fail(FIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!init) return fail(FIC_EINVAL, "init is NULL");
    if (!(tau > 0.0f) || !std::isfinite(tau)) return fail(FIC_EINVAL, "tau must be finite and > 0");
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(init[i])) return fail(FIC_EINVAL, "init[%d] is not finite", i);
    fic_mlp* M = new fic_mlp();
    M->tau = tau;
    auto bail = [&](int code) {
        fic_mlp_destroy(M);
        return code;
    };
    if (hipGetDevice(&M->device) != hipSuccess) return bail(fail(FIC_EDEVICE, "hipGetDevice failed"));
    const size_t pb = sizeof(float) * kMlpParams;
    if (hipMalloc(&M->w, pb) != hipSuccess || hipMalloc(&M->m, pb) != hipSuccess ||
        hipMalloc(&M->v, pb) != hipSuccess || hipMalloc(&M->g, pb) != hipSuccess ||
        hipMalloc(&M->w16, sizeof(_Float16) * kH16Total) != hipSuccess ||
        hipMalloc(&M->maxbits, 256) != hipSuccess)
        return bail(fail(FIC_ENOMEM, "hipMalloc of the network state failed"));
    if (hipMemcpy(M->w, init, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(M->m, 0, pb) != hipSuccess || hipMemset(M->v, 0, pb) != hipSuccess ||
        hipMemset(M->g, 0, pb) != hipSuccess)
        return bail(fail(FIC_EDEVICE, "upload of the initial parameters failed"));
    k_weights16<<<cdiv(kMlpParams, 256), 256>>>(M->w, M->w16);
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(FIC_EDEVICE, "weight conversion failed"));
    *out = M;
    return FIC_OK;
}

FIC_API int fic_mlp_destroy(fic_mlp* M) {
    if (!M) return FIC_OK;
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)M->w, (void*)M->m, (void*)M->v, (void*)M->g, (void*)M->w16, (void*)M->maxbits})
        if (p) (void)hipFree(p);
    fic::Buf* bufs[] = {&M->X, &M->H1, &M->H2, &M->Y, &M->G32, &M->nrm, &M->G16, &M->Z, &M->Pm, &M->Pt,
                        &M->GDt, &M->GRt, &M->dG, &M->dS, &M->dY, &M->D1, &M->D2, &M->T1, &M->T2,
                        &M->part, &M->sums, &M->loss, &M->keys, &M->cand, &M->fbq, &M->tmpm,
                        &M->tkq, &M->tkgm, &M->tkth, &M->tkcnt};
    for (fic::Buf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    delete M;
    return FIC_OK;
}

FIC_API int fic_mlp_get_params(const fic_mlp* M, float* out) {
    if (!M || !out) return fail(FIC_EINVAL, "NULL argument");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(out, M->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return FIC_OK;
}

FIC_API int fic_mlp_embed(fic_mlp* M, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                          int32_t kind, int32_t L, const int32_t* list, int32_t n, uint16_t* out,
                          void* stream) {
    if (!M) return fail(FIC_EINVAL, "network is NULL");
    int rc = check_block_image(img, H, W, pitch, kind == 1 ? L : 1);
    if (rc) return rc;
    if (kind != 0 && kind != 1) return fail(FIC_EINVAL, "kind %d not 0 (ranges) or 1 (domains)", kind);
    const int nd = ((H - 16) / (kind == 1 ? L : 1) + 1) * ((W - 16) / (kind == 1 ? L : 1) + 1);
    const int full = kind == 0 ? (H / 8) * (W / 8) : nd;
    if (n < 0) return fail(FIC_EINVAL, "n < 0");
    if (!list && n != full) return fail(FIC_EINVAL, "list is NULL but n %d != %d", n, full);
    if (n == 0) return FIC_OK;
    if (!out) return fail(FIC_EINVAL, "out is NULL");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("learned_embed", st);
    const int gx = (W - 16) / (kind == 1 ? L : 1) + 1;
    if ((rc = mgrow(M->X, (int64_t)n * 8 * 64 * 2))) return rc;
    k_block_rows<<<cdiv((int64_t)n * 64, 256), 256, 0, st>>>(img, pitch, H, W, kind, kind == 1 ? L : 1, gx,
                                                            nd, list, n, P<_Float16>(M->X));
    if ((rc = mlp_forward(M, n, false, st))) return rc;
    HIP_TRY(hipMemcpyAsync(out, M->G16.p, (size_t)n * 64 * 2, hipMemcpyDeviceToDevice, st));
    return FIC_OK;
}

FIC_API int fic_mlp_loss_grad(fic_mlp* M, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                              int32_t L, const int32_t* range_yx, const int32_t* labels,
                              int32_t n_ranges, float* loss_out, float* grad_out, void* stream) {
    if (!M) return fail(FIC_EINVAL, "network is NULL");
    int rc = check_block_image(img, H, W, pitch, L);
    if (rc) return rc;
    if (!labels) return fail(FIC_EINVAL, "labels is NULL");
    if (n_ranges < 1) return fail(FIC_EINVAL, "n_ranges must be >= 1");
    if (!range_yx && n_ranges != (H / 8) * (W / 8))
        return fail(FIC_EINVAL, "range_yx is NULL but n_ranges %d != %d", n_ranges, (H / 8) * (W / 8));
    hipStream_t st = (hipStream_t)stream;
    {
        ProfScope ps("learned_loss_grad", st);
        if ((rc = loss_grad_impl(M, img, H, W, pitch, L, range_yx, labels, n_ranges, loss_out, st))) return rc;
    }
    if (grad_out)
        HIP_TRY(hipMemcpyAsync(grad_out, M->g, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, st));
    return FIC_OK;
}

FIC_API int fic_mlp_adam(fic_mlp* M, const float* grad, float lr, float beta1, float beta2, float eps,
                         void* stream) {
    if (!M) return fail(FIC_EINVAL, "network is NULL");
    int rc = check_adam(lr, beta1, beta2, eps);
    if (rc) return rc;
    ProfScope ps("learned_adam", (hipStream_t)stream);
    return adam_impl(M, grad, lr, beta1, beta2, eps, (hipStream_t)stream);
}

FIC_API int fic_mlp_train_step(fic_mlp* M, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                               int32_t L, const int32_t* range_yx, const int32_t* labels,
                               int32_t n_ranges, float lr, float* loss_out, void* stream) {
    int rc = check_adam(lr, 0.9f, 0.999f, 1e-8f);
    if (rc) return rc;
    if ((rc = fic_mlp_loss_grad(M, img, H, W, pitch, L, range_yx, labels, n_ranges, loss_out, nullptr, stream)))
        return rc;
    return fic_mlp_adam(M, nullptr, lr, 0.9f, 0.999f, 1e-8f, stream);
}

FIC_API int fic_topk_similar(const uint16_t* q, int32_t nq, const uint16_t* keys, int32_t nk, int32_t k,
                             int32_t* idx, float* score, fic_mlp* M, void* stream) {
    if (!M) return fail(FIC_EINVAL, "network (scratch owner) is NULL");
    if (nq < 0 || nk < 1) return fail(FIC_EINVAL, "nq < 0 or nk < 1");
    if (k < 1 || k > kTopK) return fail(FIC_EINVAL, "k %d not in 1..%d", k, kTopK);
    if (nq == 0) return FIC_OK;
    if (!q || !keys || !idx) return fail(FIC_EINVAL, "NULL pointer");
    if (((uintptr_t)q | (uintptr_t)keys) & 15) return fail(FIC_EINVAL, "embeddings must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("learned_topk", st);
    return topk_launch(M, reinterpret_cast<const _Float16*>(q), nq, reinterpret_cast<const _Float16*>(keys), nk, k,
                       idx, score, st);
}

FIC_API int fic_encode_level_learned(fic_mlp* M, const uint8_t* img, int32_t H, int32_t W, int32_t pitch,
                                     int32_t L, const int8_t* s_k, int32_t n_s, int32_t topk,
                                     float rms_thresh, fic_match* out, int32_t* proposals_out,
                                     int32_t* n_fallback, void* stream) {
    if (!M) return fail(FIC_EINVAL, "network is NULL");
    int rc = check_block_image(img, H, W, pitch, L);
    if (rc) return rc;
    KSet ks;
    if ((rc = check_kset(s_k, n_s, &ks))) return rc;
    if (topk < 1 || topk > kTopK) return fail(FIC_EINVAL, "topk %d not in 1..%d", topk, kTopK);
    if (!(rms_thresh >= 0.0f) || !std::isfinite(rms_thresh))
        return fail(FIC_EINVAL, "rms_thresh must be finite and >= 0");
    if (!out) return fail(FIC_EINVAL, "out is NULL");
    const int nr = (H / 8) * (W / 8);
    const int gx = (W - 16) / L + 1, gy = (H - 16) / L + 1, nd = gx * gy;
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws;
    if ((rc = get_ws(st, &ws))) return rc;
    Level v = make_level(0, H, W, 8, L, nr, ks);
    Sizes sz;
    grow(sz, v);
    if ((rc = ensure_sizes(*ws, sz))) return rc;
    int32_t* act = P<int32_t>(ws->act0);
    Lvl lv = make_lvl(*ws, v, img, H, W, pitch, 0, 0.0f, 1, act, P<int32_t>(ws->act1), 1, 0, nullptr, 0, nullptr);
    if ((rc = mgrow(M->cand, (int64_t)nr * topk * 4)) || (rc = mgrow(M->fbq, (int64_t)nr * 4)) ||
        (rc = mgrow(M->tmpm, (int64_t)nr * sizeof(fic_match))))
        return rc;
    int32_t* cand = proposals_out ? proposals_out : P<int32_t>(M->cand);
    {
        ProfScope ps("learned_embed", st);
        if ((rc = block_rows(M, img, H, W, pitch, L, nullptr, nr, nd, st))) return rc;
        if ((rc = mlp_forward(M, nr + nd, false, st))) return rc;
    }
    {
        ProfScope ps("learned_topk", st);
        const _Float16* G16 = P<_Float16>(M->G16);
        if ((rc = topk_launch(M, G16, nr, G16 + (int64_t)nr * 64, nd, topk, cand, nullptr, st))) return rc;
    }
    int32_t* fb_count = ws->ctrl->act_count;  // level 0 of this workspace
    // the pool of the exhaustive fallback (every domain of the level): its
    // columns, S and A' also serve the rescoring when the level has the grid
    // matchers' layout
    std::vector<Lvl> t{lv};
    if ((rc = launch_pool_phase(nullptr, t, ws->T, false, st))) return rc;
    {
        ProfScope ps("learned_rescore", st);
        if (lv.var == kVarMfma)
            k_rescore<1><<<nr, kRsThreads, 0, st>>>(img, pitch, W, L, gx, nd, lv.dh, lv.sd, lv.ad, cand, topk, nr, ks, out);
        else
            k_rescore<0><<<nr, kRsThreads, 0, st>>>(img, pitch, W, L, gx, nd, nullptr, nullptr, nullptr, cand, topk, nr,
                                             ks, out);
        k_fallback_list<<<1, 1024, 0, st>>>(out, nr, W, keep_threshold(rms_thresh, 8), act, P<int32_t>(M->fbq),
                                            fb_count);
        LAUNCH_CHECK();
    }
    // exhaustive search for the ranges on the fallback list, each range's
    // bound started at its rescored match
    t[0].gbseed = out;
    if ((rc = launch_match_phase(nullptr, t, st))) return rc;
    {
        ProfScope ps("learned_fallback", st);
        fic_match* tmp = P<fic_match>(M->tmpm);
        kt_reduce_level<false><<<cdiv(nr, kBlock), kBlock, 0, st>>>(lv, nullptr, tmp);
        k_fallback_scatter<<<cdiv(nr, kBlock), kBlock, 0, st>>>(tmp, P<int32_t>(M->fbq), fb_count, out);
        LAUNCH_CHECK();
    }
    if (n_fallback) HIP_TRY(hipMemcpyAsync(n_fallback, fb_count, sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return FIC_OK;
}

FIC_API int fic_level_codes(const fic_match* m, int32_t H, int32_t W, int32_t B, int32_t L, fic_code* codes,
                            void* stream) {
    if (!m || !codes) return fail(FIC_EINVAL, "NULL pointer");
    if (!valid_B(B) || H < 2 * B || W < 2 * B || H % B || W % B)
        return fail(FIC_EINVAL, "image %dx%d and range side %d do not form a level", H, W, B);
    if (L < 1) return fail(FIC_EINVAL, "domain step L=%d < 1", L);
    const int nr = (H / B) * (W / B);
    const int gx = (W - 2 * B) / L + 1;
    k_level_codes<<<cdiv(nr, 256), 256, 0, (hipStream_t)stream>>>(m, nr, W, B, L, gx, codes);
    LAUNCH_CHECK();
    return FIC_OK;
}
