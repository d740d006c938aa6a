/* iga_nn.h -- C ABI of the learned preconditioner (gfx950).
 *
 * A small convolutional network on the tensor grid of one component grid
 * replaces part of the work of the fast-diagonalisation preconditioner inside
 * flexible CG.  The network: nlayers 3x3x3 convolutions with zero padding
 * ("same" size) and ReLU between layers, channels[0..nlayers].  Its input has
 * three channels, (r / ||r||, z_FD / s, log a - mean log a) with s = ||z_FD||,
 * the residual r, the fast-diagonalisation output z_FD = P^-1 r and the
 * coefficient a at the Greville points of the unknowns; its single output
 * channel y corrects z_FD: additively, z = z_FD + s y (head 0), or as a
 * log-scale, z = z_FD exp(y) (head 1).  It is trained on pairs (r, e) with
 * A e = r taken from the iterates of the plain preconditioned CG, by
 * minimising the squared error of the predicted z / s against e / s.
 *
 * Layouts: tensors [batch][channel][n3][n2][n1] (direction 1 fastest, FP32);
 * parameters one flat FP32 array, per layer w[c_out][c_in][3][3][3]
 * (tap t acting on the neighbour at offset t - 1 in each direction) followed
 * by b[c_out].  All pointers named *_dev are device memory owned by the
 * caller; work runs asynchronously on `stream` (a hipStream_t, NULL = default).
 * Every call returns an iga_status (see iga_sg.h) and sets
 * iga_sg_last_error() on failure; invalid sizes give IGA_ERR_INVALID_ARG.
 */
#ifndef IGA_NN_H
#define IGA_NN_H

#include <stdint.h>

#include "iga_sg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of FP32 parameters of the network (negative if the description is invalid). */
int64_t iga_nn_param_count(const int* channels, int nlayers);

/* Seeded initial parameters (host array of iga_nn_param_count floats): He
 * normal weights, std sqrt(2 / (27 c_in)), from a splitmix64 stream with the
 * given seed (Box-Muller normals), zero biases, and a zero last layer, so
 * that the untrained network leaves the fast-diagonalisation preconditioner
 * unchanged.  Deterministic on every host. */
iga_status iga_nn_init(const int* channels, int nlayers, uint64_t seed, float* params_host);

/* Write / read a network file: the magic "IGANNv01", layer count, head,
 * channels, parameter count, the FP32 parameters (host arrays) and a CRC-32
 * of all of it.  iga_nn_load checks the magic, the sizes and the checksum
 * (IGA_ERR_INVALID_ARG on any mismatch); channels may be NULL (sized
 * nlayers + 1 otherwise), params_host may be NULL to query the description
 * first, else it holds capacity floats. */
iga_status iga_nn_save(const char* path, const int* channels, int nlayers, int head, const float* params_host);
iga_status iga_nn_load(const char* path, int* channels, int* nlayers, int* head, float* params_host,
                       int64_t capacity);

/* Forward pass over nb tensors of shape n[3]: x_dev [nb][channels[0]][n] ->
 * y_dev [nb][channels[nlayers]][n].  acts_dev may be NULL, or hold
 * sum_{l=1}^{nlayers-1} nb * channels[l] * n floats that receive the hidden
 * activations (after ReLU), layer by layer, for iga_nn_backward. */
iga_status iga_nn_forward(const int* channels, int nlayers, const float* params_dev, int nb, const int* n,
                          const float* x_dev, float* acts_dev, float* y_dev, void* stream);

/* Gradient of L = sum (pred - t)^2 / (2 count) with respect to the
 * parameters, pred = y (head 0) or pred = x[:, 1] exp(y) (head 1, one output
 * channel), from the input x_dev, the hidden activations acts_dev and the
 * output y_dev of iga_nn_forward and the target t_dev ([nb][channels[nlayers]][n]).
 * grads_dev (param_count floats) is overwritten; loss_dev (one double) is
 * overwritten with L when not NULL; scratch_dev holds
 * 2 * nb * max_l channels[l] * n + 2048 floats. */
iga_status iga_nn_backward(const int* channels, int nlayers, const float* params_dev, int nb, const int* n,
                           const float* x_dev, const float* acts_dev, const float* y_dev, const float* t_dev,
                           int head, double count, float* grads_dev, double* loss_dev, float* scratch_dev,
                           void* stream);

/* One Adam step on count parameters (m_dev, v_dev: moment estimates, caller
 * initialised to zero; step counts from 1). */
iga_status iga_nn_adam(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev, int64_t count,
                       float lr, float beta1, float beta2, float eps, int step, void* stream);

/* One training pair of a component with n unknowns (n <= 65536): from FP64
 * r, z_FD, log a and the error e = xs - xk (converged minus current
 * iterate), writes x_dev [3][n] = (r / ||r||, z_FD / s, log a - mean log a)
 * and t_dev [n] = (e - z_FD) / s (head 0) or e / s (head 1), s = ||z_FD||
 * (norms of 0 taken as 1).  xs_dev may be NULL (then t_dev is not written);
 * xk_dev NULL means xk = 0. */
iga_status iga_nn_pair(const double* r_dev, const double* zfd_dev, const double* loga_dev, const double* xs_dev,
                       const double* xk_dev, int64_t n, int head, float* x_dev, float* t_dev, void* stream);

/* log a at the Greville points of the interior unknowns of component comp
 * (after iga_sg_assemble), lexicographic, direction 1 fastest. */
iga_status iga_sg_loga(iga_sg_plan plan, int comp, double* out_dev);

/* Attach the network used by learned solves (iga_sg_solve_opts.precond = 1;
 * three-dimensional plans, three input and one output channel, at most 32
 * and 48 channels in the two hidden layers; head as in iga_nn_backward).  params_dev stays owned by the
 * caller and must stay valid while such solves run; NULL detaches. */
iga_status iga_sg_set_network(iga_sg_plan plan, const int* channels, int nlayers, const float* params_dev,
                              int head);

#ifdef __cplusplus
}
#endif
#endif
