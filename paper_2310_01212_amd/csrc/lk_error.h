/*
 * lk_error.h -- the calling thread's last error detail, shared by every part of the host
 * library so that lk_last_error() reports failures of any exported call.
 */
#ifndef LK_ERROR_H
#define LK_ERROR_H

namespace lkh {

// Replace the calling thread's last error detail (read by lk_last_error).
void set_last_error(const char *msg);

}  // namespace lkh

#endif
