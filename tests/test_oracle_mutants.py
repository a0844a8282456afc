"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/pr_oracle.c, plants one plausible mistake (a dropped
term, a wrong sign or index, a swapped operand), builds the copy with gcc and
runs tests/test_oracle_pins.py, tests/test_oracle_display_pins.py,
tests/test_oracle_shading_pins.py and tests/test_oracle_profile_pins.py
against it; the pins must fail.  Runs on the
CPU only.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, 'oracle', 'pr_oracle.c')

MUTANTS = {
    'time_swapped_in_lerp': ('(1.0 - t) * c->Ps[3 * v + d] + t * c->Pe[3 * v + d]',
                             't * c->Ps[3 * v + d] + (1.0 - t) * c->Pe[3 * v + d]'),
    'rolling_time_unscaled': ('vp[ORC_ROLL] * (x[0] + 1.0) * 0.5', 'vp[ORC_ROLL] * (x[0] + 1.0)'),
    'foveation_exponent': ('pow(rho / orc_fovea_radius(vp), vp[ORC_ALPHA] - 1.0)', 'pow(rho / orc_fovea_radius(vp), vp[ORC_ALPHA])'),
    'foveation_radius_nearest_corner': ('if (d > best) best = d;', 'if (best == 0 || d < best) best = d;'),
    'one_sided_inside_test': ('int neg = e[0] <= 0 && e[1] <= 0 && e[2] <= 0;', 'int neg = 0;'),
    'depth_is_distance': ('*z = D / S;', '*z = D / S * norm3(r);'),
    'pixel_centre_offset': ('y[0] = 2.0 * (i + 0.5) / W - 1.0;', 'y[0] = 2.0 * (i + 1.0) / W - 1.0;'),
    'rows_not_flipped': ('y[1] = 1.0 - 2.0 * (j + 0.5) / H;', 'y[1] = 2.0 * (j + 0.5) / H - 1.0;'),
    'tie_to_higher_index': ('if (z < bz) {', 'if (z <= bz) {'),
    'rodrigues_transposed': ('double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};',
                             'double K[9] = {0, w[2], -w[1], -w[2], 0, w[0], w[1], -w[0], 0};'),
    'principal_point_sign': ('r[0] = (x[0] - vp[ORC_CX]) / vp[ORC_FX];', 'r[0] = (x[0] + vp[ORC_CX]) / vp[ORC_FX];'),
    'ambient_not_scaled': ('double s = light[3] + (1.0 - light[3]) * (ndl > 0 ? ndl : 0.0);',
                           'double s = light[3] + (ndl > 0 ? ndl : 0.0);'),
    'light_not_rolling': ('for (int d = 0; d < 3; ++d) L[d] = (1.0 - t) * l0[d] + t * l1[d];',
                          'for (int d = 0; d < 3; ++d) L[d] = l0[d];'),
    'normal_not_flipped': ('    if (dot3(n, r) > 0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }\n    double l0[3]',
                           '    double l0[3]'),
    'grad_end_weight': ('mPe[3 * (size_t)tv[k] + d] += t * gP[k][d];',
                        'mPe[3 * (size_t)tv[k] + d] += (1.0 - t) * gP[k][d];'),
    'grad_cross_order': ('cross3(P[ib], g, ta);', 'cross3(g, P[ib], ta);'),
    'grad_light_weight': ('mR[9 + 3 * rr + cc] += t * gLw[rr] * light[cc];', 'mR[9 + 3 * rr + cc] += gLw[rr] * light[cc];'),
    'grad_rotation_jacobian': ('for (int k = 0; k < 9; ++k) out[k] = Ei[k] + 0.5 * (A[k] + B[k]);',
                               'for (int k = 0; k < 9; ++k) out[k] = Ei[k];'),
    'grad_translation': ('gT0[rr] += gs_[rr];', 'gT0[rr] -= gs_[rr];'),
    'ehat_not_normalised': ('double v = cn > 0 ? fabs(e[k]) / (rn * cn) : 0.0;',
                            'double v = cn > 0 ? fabs(e[k]) / cn : 0.0;'),
    'cosinc_not_normalised': ('cosinc[q] = nn > 0 ? fabs(dot3(N, r)) / nn : 0.0;',
                              'cosinc[q] = nn > 0 ? fabs(dot3(N, r)) / norm3(N) : 0.0;'),
    # the bound invariant's checker: every hit, occluded or not
    'all_hits_first_only': ('out_ehat[count] = eh; }\n            ++count;',
                            'out_ehat[count] = eh; }\n            ++count;\n            break;'),
    'all_hits_position_not_pixel': ('if (count < cap) { out_pix[count] = p;', 'if (count < cap) { out_pix[count] = q;'),
    # the grid render
    'fast_box_start_vertices_only': ('for (int i = 0; i < 6; ++i) {\n            double q[2]',
                                     'for (int i = 0; i < 3; ++i) {\n            double q[2]'),
    'fast_near_plane_crossing_culled': ('if (n_in < 6) { kind[f] = 2; ++nglob; continue; }',
                                        'if (n_in < 6) { kind[f] = 0; continue; }'),
    'fast_tie_to_higher_index': ('if (z < *bz || (z == *bz && f < *bid)) {', 'if (z < *bz || (z == *bz && f > *bid)) {'),
    'fast_cell_axes_swapped': ('size_t c = (size_t)grid_cell(x[1], g) * g + grid_cell(x[0], g);',
                               'size_t c = (size_t)grid_cell(x[0], g) * g + grid_cell(x[1], g);'),
    # rolling highlight and G-buffer
    'highlight_eye_sign': ('if (ks == 0.0 || dot3(n, l) <= 0.0) return 0.0;\n    double rn = norm3(r);',
                           'if (ks == 0.0 || dot3(n, l) <= 0.0) return 0.0;\n    double rn = -norm3(r);'),
    'highlight_not_gated': ('if (ks == 0.0 || dot3(n, l) <= 0.0) return 0.0;', 'if (ks == 0.0) return 0.0;'),
    'highlight_exponent': ('return ndh > 0.0 ? ks * pow(ndh, m) : 0.0;', 'return ndh > 0.0 ? ks * pow(ndh, m - 1.0) : 0.0;'),
    'highlight_half_vector_unnormalised': ('double ndh = dot3(n, H) / hn;', 'double ndh = dot3(n, H);'),
    'highlight_eye_unnormalised': ('    double H[3] = {l[0] - r[0] / rn, l[1] - r[1] / rn, l[2] - r[2] / rn};\n    double hn',
                                   '    double H[3] = {l[0] - r[0], l[1] - r[1], l[2] - r[2]};\n    double hn'),
    'grad_highlight_normal_dropped': ('gn[d] += gsig * h[d];', 'gn[d] += 0.0 * h[d];'),
    'grad_highlight_light_dropped': ('gl[d] += (gh[d] - h[d] * hg) / hn;', 'gl[d] += gh[d] / hn;'),
    'gbuffer_bary_vertex': ('out_bary[2 * q] = mu[1];', 'out_bary[2 * q] = mu[0];'),
    'gbuffer_normal_not_flipped': ('            if (dot3(n, r) > 0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }\n        }',
                                   '        }'),
    'gbuffer_density_not_sqrt': ('out_density[q] = sqrt(fabs(JF[0] * JF[3] - JF[1] * JF[2]));',
                                 'out_density[q] = fabs(JF[0] * JF[3] - JF[1] * JF[2]);'),
    'gbuffer_density_display_distance': ('orc_foveate_jac(vp, xp, JF);\n        out_density',
                                         'orc_foveate_jac(vp, y, JF);\n        out_density'),
    # tabulated foveation and lens distortion
    'tab_inverse_segment': ('while (k < n - 2 && tab[k + 1] <= u) ++k;', 'while (k < n - 2 && tab[k] <= u) ++k;'),
    'tab_eval_segment_offset': ('return tab[k] + (s - k * h) / h * (tab[k + 1] - tab[k]);',
                                'return tab[k] + s / h * (tab[k + 1] - tab[k]);'),
    'tab_slope_not_scaled': ('return (tab[k + 1] - tab[k]) / h;', 'return (tab[k + 1] - tab[k]);'),
    'tab_unfoveate_uses_power_law': ('double s = vp[ORC_NC] > 0 ? tab_scale(vp, 0, 1, rho) :',
                                     'double s = 0 ? tab_scale(vp, 0, 1, rho) :'),
    'lens_not_applied': ('    orc_undistort(vp, xp, x);\n    r[0]', '    x[0] = xp[0]; x[1] = xp[1];\n    r[0]'),
    'lens_forward_not_inverse': ('double s = tab_scale(vp, 1, 1, rho);', 'double s = tab_scale(vp, 1, 0, rho);'),
    'time_from_undistorted_point': ('*t = orc_pixel_time(vp, xp);\n    orc_undistort(vp, xp, x);',
                                    'orc_undistort(vp, xp, x);\n    *t = orc_pixel_time(vp, x);'),
    'tab_jacobian_radial_dropped': ('(gp - gs) * d[r] * d[c] / rho2', '0.0 * d[r] * d[c] / rho2'),
    # display unfoveation
    'mip_texel_centre_shift': ('double uk0 = (u[0] + 0.5) * sc - 0.5, uk1 = (u[1] + 0.5) * sc - 0.5;',
                               'double uk0 = u[0] * sc, uk1 = u[1] * sc;'),
    'mip_box_mean_weight': ('dst[4 * ((size_t)j * w + i) + c] = 0.25 * s;', 'dst[4 * ((size_t)j * w + i) + c] = 0.3 * s;'),
    'mip_odd_edge_wraps': ('if (ii > pw - 1) ii = pw - 1;', 'if (ii > pw - 1) ii = 0;'),
    'lod_shorter_column': ('double l = c0 > c1 ? c0 : c1;', 'double l = c0 < c1 ? c0 : c1;'),
    'catmull_rom_weight': ('w[1] = 0.5 * (2 - 5 * t * t + 3 * t * t * t);', 'w[1] = 0.5 * (2 - 4 * t * t + 3 * t * t * t);'),
    'level_blend_reversed': ('out[c] = (1.0 - fr) * a[c] + fr * b[c];', 'out[c] = fr * a[c] + (1.0 - fr) * b[c];'),
    'filter_distance_foveated': ('orc_unfoveate(vp, yv, xv);', 'xv[0] = yv[0]; xv[1] = yv[1];'),
    'unfov_jacobian_sign': ('(e - 1.0) * s * d[r] * d[c] / rho2', '(1.0 - e) * s * d[r] * d[c] / rho2'),
    'unfov_row_not_flipped': ('u[1] = (1.0 - y[1]) * 0.5 * H - 0.5;', 'u[1] = (y[1] + 1.0) * 0.5 * H - 0.5;'),
}


def _run(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f'{name}: pattern must occur exactly once'
    d = os.path.join(tmp, name)
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, 'm.c')
    so = os.path.join(d, 'm.so')
    open(c, 'w').write(src.replace(old, new))
    subprocess.check_call(['gcc', '-O2', '-fopenmp', '-fPIC', '-shared', '-std=c11', '-o', so, c, '-lm'])
    env = dict(os.environ, PR_ORACLE_LIB=so, OMP_NUM_THREADS='2')
    r = subprocess.run([sys.executable, '-m', 'pytest', '-x', '-q', '-p', 'no:cacheprovider',
                        os.path.join(ROOT, 'tests', 'test_oracle_pins.py'),
                        os.path.join(ROOT, 'tests', 'test_oracle_display_pins.py'),
                        os.path.join(ROOT, 'tests', 'test_oracle_shading_pins.py'),
                        os.path.join(ROOT, 'tests', 'test_oracle_profile_pins.py')],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda n: _run(n, str(tmp_path)), sorted(MUTANTS)))
    survived = [n for n, rc in results if rc == 0]
    assert not survived, f'mutants not caught by the pins: {survived}'
