// Workspace sizing of every entry point (dry runs of the same arena layouts
// the calls use).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace xtc {
size_t ws_eval_orbitals(int64_t n_g, int n_orb, int n_ao);
size_t ws_select(int64_t n_g, int n_orb, int n_mu, int mode);
size_t ws_fit(int64_t n_g, int n_orb, int n_mu, uint32_t what);
size_t ws_contract(int64_t n_g, int n_mu, uint32_t flags, int n_orb, int n_q);
size_t ws_grad(int64_t n_g, int n_mu, int n_params, uint32_t flags);
size_t ws_features(int64_t n_g);
size_t ws_mlp_grad(int64_t n, int hidden);
size_t ws_learned(int64_t n_g, int n_orb, int n_mu, double kappa, long stride);
size_t ws_fit_residual(int64_t n_g, int n_orb, int n_mu);
size_t ws_exchange(int64_t n_g, int n_orb, int n_mu, int n_q, int precision);
size_t ws_assembly(int n_orb, int n_mu, uint32_t outputs);
size_t ws_one_body(int n_orb, int n_mu);
size_t ws_vmc(int n_ao);
}  // namespace xtc
